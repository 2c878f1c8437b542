// Host side of libmg: argument checks, level hierarchies, cycle programs, the
// solve loops and the C ABI declared in include/mg.h.
//
// The cycle is compiled once, at setup, into a flat list of ops by walking
// the recursive algorithm MG(l, u, g) ("The Multigrid Technique"): smoothing,
// defect restriction, the recursive coarse calls (an F-cycle gives the coarse
// problem one F-cycle then one V-cycle), prolongation with omega_l = 1 and the
// exact coarsest solve.  Large levels run as fused LDS-tiled passes; small
// levels run their whole sub-cycle in one launch of a single-workgroup
// kernel.  The cycle is captured as a HIP graph; the solve loop replays it in
// batches and reads the device-side stopping state once per batch.
//
// A handle holds one or more groups.  A group is a set of problems with the
// same grid (the batched solver groups its problems by grid); all of a
// group's problems go through the same launches, one problem per blockIdx.z,
// each masked once its own stopping test is met.  The groups of a batched
// handle are captured as parallel branches of one graph.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "mg.h"
#include "mg_fused.h"
#include "mg_kernels.h"
#include "mg_tune.h"

using namespace mg;

namespace {

thread_local std::string g_thread_err;

constexpr int MAX_BATCH = 4096;

enum HostOpType {
  H_COLOR = 0, H_JACOBI, H_COPY, H_DR, H_PROLONG, H_COARSE, H_SUB, H_PRE, H_POST, H_LINE, H_OMEGA,
  H_NORM  // merged batched schedule: stopping test of the problems whose cycle just ended
};

struct HostOp {
  int type, level, arg;
  int sub;  // H_SUB: index of its device sub-program
};

struct Abs {  // abstract op of the expanded cycle
  int type, level, arg;
};

int round_up(int v, int m) { return (v + m - 1) / m * m; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Problems of one grid.  Level descriptors are kept twice on the device:
// level-major [level][slot] for per-op and tile kernels (blockIdx.z = slot)
// and problem-major [slot][level] for the coarse-level kernel.
struct Group {
  int ns = 1;
  std::vector<int> probs;  // problem index of each slot
  mg_grid grid{};
  int nlev = 0, ncu = 0;
  int threshold = 0;  // coarse-level kernel: levels of at most this many nodes (0: those whose sub-hierarchy fits LDS)
  std::vector<LevelShape> shp;
  std::vector<double> hx, hy;
  std::vector<Level<double>> L64;  // [level * ns + slot]
  std::vector<Level<float>> L32;
  Level<double>* dL64 = nullptr;
  Level<float>* dL32 = nullptr;
  Level<double>* dP64 = nullptr;
  Level<float>* dP32 = nullptr;
  std::vector<double*> band64;
  std::vector<float*> band32;
  double** dcholp = nullptr;  // inverse of each slot's coarsest operator
  std::vector<double*> chol, cinv;  // per slot: coarsest dense matrix / Cholesky factor, its inverse
  int* dinfo = nullptr;             // per slot: Cholesky status
  std::vector<TileGeom> gpre, gpost;
  bool norm_fused = false;   // FP64: the finest post-pass applies the stopping test
  bool mixed_fused = false;  // mixed: the finest post-pass adds e into the FP64 iterate
  bool resid_kernel = false;  // mixed: keep the residual kernel where the pre-pass could form r (tuned)
  std::vector<HostOp> prog;
  DOp* dprog = nullptr;
  int* dbeg = nullptr;  // [sub * ns + slot]
  int* dcnt = nullptr;
  int nsub = 0;
  hipStream_t branch = nullptr;  // capture branch of this group

  Level<double>& l64(int l, int s) { return L64[(size_t)l * ns + s]; }
  Level<float>& l32(int l, int s) { return L32[(size_t)l * ns + s]; }
  const Level<double>& l64(int l, int s) const { return L64[(size_t)l * ns + s]; }
};

// Batched problems whose level chains end alike (each group's level shapes
// are the last ones of the deepest group's) run one merged schedule: the
// deepest group's cycle, in which every smaller group takes part in exactly
// the recursive call that is its own cycle (the first call on its finest
// level), each launch covering every problem on that level through a table
// of their level descriptors.
struct MOp {
  int type = 0, level = 0, arg = 0;  // as HostOp; level counts on the deepest chain
  int fine = 0;                      // the participants are on their finest level
  int tab = -1, ctab = -1;           // descriptor tables of `level` and `level + 1` (H_SUB: problem-major)
  int n = 0;                         // participants
  int* dbeg = nullptr;               // H_SUB: per participant, the sub-program's begin and count
  int* dcnt = nullptr;
  double** dchol = nullptr;          // H_SUB: per participant, its coarsest inverse
  TileGeom g{};                      // H_PRE, H_POST
};

struct MTab {
  std::vector<std::array<int, 3>> mem;  // (group, slot, level of that group) per entry
  Level<double>* d64 = nullptr;
  Level<float>* d32 = nullptr;
};

struct Merge {
  std::vector<int> groups;  // deepest first
  std::vector<int> off;     // per group: level of the deepest chain holding its finest level
  int nlev = 0;
  std::vector<MOp> prog;
  std::vector<MTab> tabs;
  std::map<std::string, int> tab_index;
  DOp* dprog = nullptr;     // sub-programs, levels relative to the sub-cycle's top
  hipStream_t branch = nullptr;
};

}  // namespace

struct mg_handle_s {
  bool batched = false;
  int nprob = 1;
  int kind = MG_COEF_CONST5;
  int oned = 0;                      // the hierarchy's 9-point bands vary along x only
  int in_oned = 0;                   // layout of the caller's cell arrays (kx_1d_along_x)
  // refined (graded) grid: cell widths over the equidistant ones, per cell
  // column and row (host and device), and the caller's coefficients folded
  // with them (device, `grows` rows of ncx)
  bool graded = false;
  std::vector<double> hrx, hry;
  double *grx = nullptr, *gry = nullptr, *gkx = nullptr, *gky = nullptr;
  int grows = 1;
  bool galerkin5 = false;            // 5-point problem with Galerkin coarse operators (levels kept as 1-D bands)
  mg_options opts{};
  int ncol = 0;                      // 0 Jacobi (and line smoothers), 2 red-black, 4 four-colour
  int line = 0;                      // line smoothers: directions swept (bit 0 x, bit 1 y)
  bool line_jac = false;             // line smoothers: Jacobi (TRI) rather than Gauss-Seidel
  std::vector<double> eps_x, eps_y;  // per problem (5-point)
  int* dcount = nullptr;             // cell coefficients: count of invalid values (setup and update)
  hipStream_t stream = nullptr;
  int ncus = 256;                    // compute units of the device (workgroups that fill it once)
  std::string err;

  std::vector<Group> groups;
  std::vector<Merge> merges;      // batched: merged schedules
  std::vector<int> standalone;    // batched: groups that run their own cycle (branch)

  // device memory
  std::vector<void*> allocs;
  SolveState* dstate = nullptr;      // [nprob]
  SolveState* dstate_res = nullptr;  // mg_residual's own state
  Level<double>* dLres = nullptr;    // mg_residual's finest-level descriptor
  std::vector<double*> dhist;        // per problem
  int hist_cap = 0;
  std::vector<double*> dpartial;     // per problem
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<hipEvent_t> fork;      // capture fork/join events

  // one cycle and eight cycles captured as graphs (kernel nodes only)
  hipStream_t cap = nullptr;
  hipGraphExec_t g1 = nullptr, g8 = nullptr;
  int graph_nodes = 0;  // nodes (launches) of the one-cycle graph

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

int stencil_kind(mg_handle h) { return (h->kind == MG_COEF_CONST5 && !h->galerkin5) ? ST5 : ST9; }

// FP32 cycles of one mixed-precision outer step (option inner_cycles, 0 = 1).
int inner_cycles(mg_handle h) { return h->opts.inner_cycles > 0 ? h->opts.inner_cycles : 1; }

// ----------------------------------------------------------------------- cycle program

// Bytes of LDS that levels l..L-1 need inside the coarse-level kernel.
size_t sub_footprint(mg_handle h, const Group& G, int l) {
  const size_t elem = h->mixed() ? sizeof(float) : sizeof(double);
  const size_t narr = h->ncol == 0 ? 3 : 2;
  const bool bands = stencil_kind(h) == ST9 && h->oned;  // 1-D bands staged in LDS too
  size_t n = 0;
  for (int k = l; k < G.nlev; ++k) n += (size_t)G.shp[k].nx * G.shp[k].ny * narr + (bands ? NBANDS * G.shp[k].nx : 0);
  if (h->line) n += 4 * (size_t)(G.shp[l].nx - 2) * G.shp[l].nrows;  // line-sweep scratch (largest level)
  return n * elem;
}

struct Gen {
  mg_handle h;
  const Group& G;
  int threshold;  // 0: the largest levels whose sub-hierarchy fits in LDS
  bool small(int l) const {
    const LevelShape& s = G.shp[l];
    if (threshold > 0) return (long)s.nx * s.ny <= threshold;
    return sub_footprint(h, G, l) <= SUB_LDS_BUDGET;
  }
  void smooth(std::vector<Abs>& out, int l, int steps) const {
    if (h->line) {
      int par = 0;  // Jacobi ping-pong: 0 x -> t, 1 t -> x
      for (int s = 0; s < steps; ++s)
        for (int dir = 0; dir < 2; ++dir) {
          if (!((h->line >> dir) & 1)) continue;
          if (h->line_jac) {
            out.push_back({H_LINE, l, line_arg(dir, true, par)});
            par ^= 1;
          } else {
            out.push_back({H_LINE, l, line_arg(dir, false, 0)});
            out.push_back({H_LINE, l, line_arg(dir, false, 1)});
          }
        }
      if (par) out.push_back({H_COPY, l, 0});
      return;
    }
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
    if (l == G.nlev - 1) {
      if (out.empty() || out.back().type != H_COARSE) out.push_back({H_COARSE, l, 0});
      return;
    }
    smooth(out, l, h->opts.nu_pre);
    out.push_back({H_DR, l, 0});
    if (kind == MG_CYCLE_F) {
      expand(out, l + 1, MG_CYCLE_F);
      expand(out, l + 1, MG_CYCLE_V);
    } else if (kind == MG_CYCLE_W) {
      expand(out, l + 1, MG_CYCLE_W);
      expand(out, l + 1, MG_CYCLE_W);
    } else {
      expand(out, l + 1, MG_CYCLE_V);
    }
    if (h->opts.adaptive_omega) out.push_back({H_OMEGA, l, 0});  // omega_l from x (the smoothed iterate)
    out.push_back({H_PROLONG, l, h->opts.adaptive_omega ? 1 : 0});
    smooth(out, l, h->opts.nu_post);
  }
  // Host program: ops on large levels, one H_SUB per maximal small-level call.
  void host(std::vector<HostOp>& out, std::vector<std::vector<Abs>>& subs, int l, int kind) const {
    if (small(l) || l == G.nlev - 1) {
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
    const bool fused = h->opts.tile_mode != MG_TILES_PER_OP && !h->line;
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
    } else if (kind == MG_CYCLE_W) {
      host(out, subs, l + 1, MG_CYCLE_W);
      host(out, subs, l + 1, MG_CYCLE_W);
    } else {
      host(out, subs, l + 1, MG_CYCLE_V);
    }
    if (fused) {
      // omega_l from t, where the fused pre-pass left the smoothed iterate;
      // the post-pass applies it (the level's descriptor carries the weight)
      if (h->opts.adaptive_omega) out.push_back({H_OMEGA, l, 1, -1});
      out.push_back({H_POST, l, POST_PLAIN, -1});
      return;
    }
    if (h->opts.adaptive_omega) out.push_back({H_OMEGA, l, 0, -1});
    out.push_back({H_PROLONG, l, h->opts.adaptive_omega ? 1 : 0, -1});
    tmp.clear();
    smooth(tmp, l, h->opts.nu_post);
    for (const Abs& a : tmp) out.push_back({a.type, a.level, a.arg, -1});
  }
};

// Relaxation factor the smoothing kernels receive: the SOR factor for the
// point Gauss-Seidel smoothers (0 stands for 1), omega for the others.
double relax(mg_handle h) {
  if (h->ncol > 0) return h->opts.sor == 0.0 ? 1.0 : h->opts.sor;
  return h->opts.omega;
}

// Halo of a fused pass: one node per colour sweep (or Jacobi step), plus 2
// for the defect and its restriction (pre) or 1 for the residual (post).
int sweeps(mg_handle h, int steps) { return h->ncol == 0 ? steps : steps * h->ncol; }

// Row halo of a wide-tile pass whose column halo is H: with four colours the
// stale rows advance one per two colour steps (wrow_shrink in
// mg_fused.hip), so the sweeps need half their steps in rows; the rest of H
// (defect and restriction rows of a pre-pass, the residual's ring of a
// post-pass) carries over.  Other smoothers: H.
int row_halo(mg_handle h, int H, bool post) {
  if (h->ncol != 4) return H;
  const int steps = sweeps(h, post ? h->opts.nu_post : h->opts.nu_pre);
  return (steps + 1) / 2 + (H - steps);
}

TileGeom choose_tile_for(mg_handle h, const LevelShape& s, int ns, int H, bool post) {
  const long CHIP_CUS = h->ncus;  // workgroups that fill the chip once
  const size_t elem = h->mixed() ? sizeof(float) : sizeof(double);
  const int narr = h->ncol == 0 ? 3 : 2;
  auto bytes = [&](int TX, int TY) {
    const size_t W = TX + 2 * H, R = TY + 2 * H;
    size_t n = W * R * narr + NBANDS * W;  // + LDS copy of 1-D bands
    if (post) n += ((W >> 1) + 2) * ((R >> 1) + 2);
    return n * elem;
  };
  const bool fixed = h->opts.tile_x > 0 && h->opts.tile_y > 0;
  int TX = h->opts.tile_x > 0 ? h->opts.tile_x : 64;
  int TY = h->opts.tile_y > 0 ? h->opts.tile_y : 32;
  // tiles over all of the group's problems
  auto ntiles = [&](int tx, int ty) { return (long)ns * ((s.nx + tx - 1) / tx) * ((s.ny + ty - 1) / ty); };
  // wide tiles (fixed region width, output width WW - 2H) wherever they
  // still give the chip enough workgroups; at most WIDE_LDS_TARGET of LDS so
  // that two workgroups share a CU
  const int mode = h->opts.tile_mode;
  if (mode != MG_TILES_NARROW && h->opts.tile_x == 0 && H <= 24) {
    const int WW = wide_width(), TXw = WW - 2 * H, Hy = row_halo(h, H, post);
    auto wbytes = [&](int ty) {
      const size_t R = ty + 2 * Hy;
      size_t n = R * narr * WW + NBANDS * WW;
      if (post) n += (size_t)(WW / 2 + 2) * ((R >> 1) + 2);
      return n * elem;
    };
    const bool force = mode == MG_TILES_WIDE;
    // FP32: up to 32 rows within WIDE_LDS_TARGET (two workgroups per CU);
    // FP64: up to 40 rows in one workgroup's LDS (taller tiles, less halo,
    // measured faster than two shorter tiles per CU)
    const size_t cap = elem == sizeof(float) ? WIDE_LDS_TARGET : FUSED_LDS_MAX;
    int TYw = h->opts.tile_y > 0 ? h->opts.tile_y : (elem == sizeof(float) ? 32 : 40);
    if (h->opts.tile_y == 0)
      while (TYw > (force ? 2 : 16) && ((!force && ntiles(TXw, TYw) < CHIP_CUS) || wbytes(TYw) > cap)) TYw -= 2;
    // Between one and two tiles per CU, the CUs that get a second tile (run
    // beside the first or after it) set the pass time: the smallest taller
    // tile that leaves at most one per CU is faster while its region grows by
    // at most a quarter (1025^2: FP32 post-pass 13.6 -> 12.1 us, FP64 20.6
    // -> 13.6 us).
    if (h->opts.tile_y == 0 && !force) {
      const long nt = ntiles(TXw, TYw);
      if (nt > CHIP_CUS && nt <= 2 * CHIP_CUS)
        for (int ty = TYw + 2; 4 * (ty + 2 * Hy) <= 5 * (TYw + 2 * Hy) && wbytes(ty) <= FUSED_LDS_MAX; ty += 2)
          if (ntiles(TXw, ty) <= CHIP_CUS) return wide_geom(s.nx, s.ny, ty, H, Hy);
    }
    if ((force || ntiles(TXw, TYw) >= CHIP_CUS) && wbytes(TYw) <= FUSED_LDS_MAX)
      return wide_geom(s.nx, s.ny, TYw, H, Hy);
  }
  if (!fixed) {
    while (ntiles(TX, TY) < CHIP_CUS && TY > 8) TY >>= 1;
    while (ntiles(TX, TY) < CHIP_CUS && TX > 16) TX >>= 1;
    // as for wide tiles: at most one tile per CU when there are between one
    // and two per CU (513^2: 297 -> 234 tiles of 64 x 20)
    const long nt = ntiles(TX, TY);
    if (h->opts.tile_y == 0 && nt > CHIP_CUS && nt <= 2 * CHIP_CUS)
      for (int ty = TY + 2; 4 * (ty + 2 * H) <= 5 * (TY + 2 * H) && bytes(TX, ty) <= FUSED_LDS_MAX; ty += 2)
        if (ntiles(TX, ty) <= CHIP_CUS) {
          TY = ty;
          break;
        }
  }
  while (bytes(TX, TY) > FUSED_LDS_MAX && TY > 2) TY >>= 1;
  while (bytes(TX, TY) > FUSED_LDS_MAX && TX > 2) TX >>= 1;
  return tile_geom(s.nx, s.ny, TX, TY, H);
}

TileGeom choose_tile(mg_handle h, const Group& G, int l, int H, bool post) {
  return choose_tile_for(h, G.shp[l], G.ns, H, post);
}

// Coarse-level kernel ops from flat[b] on: runs of Gauss-Seidel colour ops
// that form whole sweeps of one level (colours 0 .. ncol - 1, repeated)
// become one OP_SMOOTH op whose arg is the number of sweeps.
void fold_sweeps(std::vector<DOp>& flat, size_t b, int ncol) {
  if (ncol <= 0) return;
  std::vector<DOp> out(flat.begin(), flat.begin() + b);
  for (size_t k = b; k < flat.size();) {
    size_t q = k;
    while (q < flat.size() && flat[q].type == OP_COLOR && flat[q].level == flat[k].level &&
           flat[q].arg == (int)((q - k) % ncol))
      ++q;
    const int sweeps = (int)std::min<size_t>((q - k) / ncol, SM_NSW);
    if (sweeps > 0) {
      out.push_back({OP_SMOOTH, flat[k].level, sweeps, 0});
      k += (size_t)sweeps * ncol;
    } else {
      out.push_back(flat[k]);
      ++k;
    }
  }
  flat.swap(out);
}

// Transfers folded into the smoothing blocks beside them (ops from flat[b]
// on): a prolongation followed by a block on its level becomes that block's
// SM_PRO (SM_WTD when weighted by omega_l); a block followed by a
// restriction of its level takes SM_DR.
void fold_transfers(std::vector<DOp>& flat, size_t b) {
  std::vector<DOp> out(flat.begin(), flat.begin() + b);
  for (size_t k = b; k < flat.size(); ++k) {
    const DOp& o = flat[k];
    if (o.type == OP_PROLONG && k + 1 < flat.size() && flat[k + 1].type == OP_SMOOTH &&
        flat[k + 1].level == o.level && !(flat[k + 1].arg & SM_PRO)) {
      DOp sm = flat[k + 1];
      sm.arg |= SM_PRO | (o.arg ? SM_WTD : 0);
      out.push_back(sm);
      ++k;
      continue;
    }
    if (o.type == OP_DR && out.size() > b && out.back().type == OP_SMOOTH && out.back().level == o.level &&
        !(out.back().arg & SM_DR)) {
      out.back().arg |= SM_DR;
      continue;
    }
    out.push_back(o);
  }
  flat.swap(out);
}

mg_status build_program(mg_handle h, Group& G) {
  Gen g{h, G, G.threshold};
  std::vector<std::vector<Abs>> subs;
  G.prog.clear();
  g.host(G.prog, subs, 0, h->opts.cycle);
  G.gpre.assign(G.nlev, TileGeom{});
  G.gpost.assign(G.nlev, TileGeom{});
  G.norm_fused = G.mixed_fused = false;
  if (!G.prog.empty() && G.prog.back().type == H_POST && G.prog.back().level == 0) {
    if (h->mixed()) {
      G.prog.back().arg = POST_MIXED;
      G.mixed_fused = true;
    } else {
      G.prog.back().arg = POST_NORM;
      G.norm_fused = true;
    }
  }
  for (const HostOp& op : G.prog) {
    if (op.type == H_PRE) G.gpre[op.level] = choose_tile(h, G, op.level, sweeps(h, h->opts.nu_pre) + 2, false);
    if (op.type == H_POST)
      G.gpost[op.level] =
          choose_tile(h, G, op.level, sweeps(h, h->opts.nu_post) + (op.arg == POST_NORM ? 1 : 0), true);
  }
  std::vector<DOp> flat;
  std::vector<int> beg, cnt;
  for (const auto& s : subs) {
    const int b = (int)flat.size();
    for (int k = 0; k < G.ns; ++k) {  // every slot of a group runs the same program
      beg.push_back(b);
      cnt.push_back((int)s.size());
    }
    for (const Abs& a : s) {
      int t = OP_COLOR;
      switch (a.type) {
        case H_COLOR: t = OP_COLOR; break;
        case H_JACOBI: t = OP_JACOBI; break;
        case H_COPY: t = OP_COPY; break;
        case H_DR: t = OP_DR; break;
        case H_PROLONG: t = OP_PROLONG; break;
        case H_COARSE: t = OP_COARSE; break;
        case H_LINE: t = OP_LINE; break;
        case H_OMEGA: t = OP_OMEGA; break;
      }
      flat.push_back({t, a.level, a.arg, 0});
    }
    fold_sweeps(flat, (size_t)b, h->ncol);
    fold_transfers(flat, (size_t)b);
    for (size_t k = cnt.size() - G.ns; k < cnt.size(); ++k) cnt[k] = (int)(flat.size() - b);
  }
  G.nsub = (int)subs.size();
  if (!flat.empty()) {
    HIPCHK(h, h->dalloc(&G.dprog, flat.size() * sizeof(DOp)));
    HIPCHK(h, hipMemcpyAsync(G.dprog, flat.data(), flat.size() * sizeof(DOp), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, h->dalloc(&G.dbeg, beg.size() * sizeof(int)));
    HIPCHK(h, h->dalloc(&G.dcnt, cnt.size() * sizeof(int)));
    HIPCHK(h, hipMemcpyAsync(G.dbeg, beg.data(), beg.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(G.dcnt, cnt.data(), cnt.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));  // the host vectors are about to go
  }
  return MG_OK;
}

template <typename T>
hipError_t run_op(mg_handle h, const Group& G, const HostOp& op, Level<T>* dL, Level<T>* dP, T omega,
                  hipStream_t st) {
  const int l = op.level, ns = G.ns;
  const LevelShape& s = G.shp[l];
  Level<T>* Ls = dL + (size_t)l * ns;
  Level<T>* Cs = dL + (size_t)(l + 1) * ns;
  switch (op.type) {
    case H_COLOR: return launch_colour<T>(Ls, s, op.arg, h->ncol, omega, ns, st);
    case H_JACOBI: return launch_jacobi<T>(Ls, s, op.arg, omega, ns, st);
    case H_COPY: return launch_copy<T>(Ls, s, ns, st);
    case H_DR: return launch_dr<T>(Ls, Cs, G.shp[l + 1], ns, st);
    case H_PROLONG: return launch_prolong<T>(Ls, Cs, s, op.arg, ns, st);
    case H_OMEGA: return launch_energy<T>(Ls, Cs, s, op.arg, stencil_kind(h), ns, st);
    case H_COARSE: return launch_coarse<T>(Ls, G.dcholp, G.ncu, ns, st);
    case H_LINE: return launch_line<T>(Ls, s, op.arg, omega, stencil_kind(h), ns, st);
    case H_PRE:
      return launch_pre<T>(Ls, Cs, G.gpre[l], h->opts.nu_pre, h->ncol, omega, stencil_kind(h), h->oned, l == 0, ns,
                           st, op.arg, l == 0 ? G.dL64 : nullptr);
    case H_POST:
      return launch_post<T>(Ls, Cs, G.gpost[l], h->opts.nu_post, h->ncol, omega, op.arg, G.dL64, stencil_kind(h),
                            h->oned, l == 0, ns, st);
    case H_SUB: {
      const size_t bytes = sub_footprint(h, G, l);
      const int* beg = G.dbeg + (size_t)op.sub * ns;
      const int* cnt = G.dcnt + (size_t)op.sub * ns;
      if (bytes <= SUB_LDS_BUDGET)
        return launch_subcycle_lds<T>(dP, G.nlev, l, G.dprog, beg, cnt, G.dcholp, G.ncu, omega, h->ncol,
                                      h->ncol == 0 ? 3 : 2, stencil_kind(h), h->oned, bytes, ns, st);
      return launch_subcycle<T>(dP, G.nlev, G.dprog, beg, cnt, G.dcholp, G.ncu, omega, h->ncol, ns, st);
    }
  }
  return hipErrorInvalidValue;
}

// Mixed form: the first inner cycle's finest pre-pass takes e = 0 without
// reading it (so the finest post-pass need not write e = 0) when the cycle
// starts with that level's wide pre-pass and ends with its fused mixed
// post-pass (not with the adaptive weight, whose energy sums read the
// finest iterate).
bool mixed_zero_start(mg_handle h, const Group& G) {
  return h->mixed() && G.mixed_fused && !h->opts.adaptive_omega && !G.prog.empty() && G.prog[0].type == H_PRE &&
         G.prog[0].level == 0 && G.gpre[0].wide;
}

// Mixed form with a zero start whose pre-pass tile fits the residual modes:
// the first finest pre-pass of an outer step forms r = b - A x (FP64) and
// its norm itself, and the stopping test of a cycle's result is taken at
// the start of the next cycle (or by tail_check) instead of by a residual
// kernel after the cycle.
bool resid_possible(mg_handle h, const Group& G) {
  return mixed_zero_start(h, G) && pre_resid_fits(G.gpre[0]) && pre_resid_kind(stencil_kind(h), h->oned);
}
bool resid_fused(mg_handle h, const Group& G) { return resid_possible(h, G) && !G.resid_kernel; }

// The stopping test of the iterate the last queued cycle left (groups whose
// cycles test at their start): its residual norm by the finest pre-pass in
// PRE_RESID_ONLY mode, then the test, if that iterate was not tested yet.
hipError_t tail_check(mg_handle h, const Group& G, hipStream_t st) {
  const TileGeom& g = G.gpre[0];
  hipError_t e = launch_pre<float>(G.dL32, G.dL32 + 1, g, h->opts.nu_pre, h->ncol, (float)relax(h), stencil_kind(h),
                                   h->oned, true, G.ns, st, PRE_RESID_ONLY, G.dL64);
  if (e != hipSuccess) return e;
  return launch_norm_finish<double>(G.dL64, g.ntx * g.nty, NORM_LAG, G.ns, st);
}

// A wide pre-pass that directly follows the pre-pass of the next finer
// level starts from x = 0 (that pass's restriction cleared it), so it need
// not read x.
HostOp with_zero_start(const Group& G, size_t k) {
  HostOp op = G.prog[k];
  if (op.type == H_PRE && op.arg == PRE_LOAD && k > 0 && G.prog[k - 1].type == H_PRE &&
      G.prog[k - 1].level + 1 == op.level && G.gpre[op.level].wide)
    op.arg = PRE_ZERO;
  return op;
}

// One cycle of a group plus its stopping test, on stream st.
hipError_t enqueue_cycle(mg_handle h, const Group& G, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (!h->mixed()) {
    for (size_t k = 0; k < G.prog.size(); ++k)
      if ((e = run_op<double>(h, G, with_zero_start(G, k), G.dL64, G.dP64, relax(h), st)) != hipSuccess) return e;
    if (G.norm_fused) return hipSuccess;
    return launch_resnorm<double>(G.dL64, G.shp[0], NORM_CHECK, nullptr, nullptr, stencil_kind(h), h->oned, G.ns,
                                  st);
  }
  // inner FP32 cycles on A e = r32 from e = 0; only the last one adds e into
  // the FP64 iterate (the finest post-pass of the others keeps e).  When
  // the cycle starts with the finest level's wide pre-pass, the first inner
  // cycle's pre-pass takes e = 0 without reading it, so the last post-pass
  // need not write e = 0 (not with the adaptive weight, whose energy sums
  // read the finest iterate)
  const int inner = inner_cycles(h);
  const bool zero_start = mixed_zero_start(h, G);
  const bool rf = resid_fused(h, G);
  for (int c = 0; c < inner; ++c)
    for (size_t k = 0; k < G.prog.size(); ++k) {
      HostOp op = with_zero_start(G, k);
      if (G.mixed_fused && c + 1 < inner && k + 1 == G.prog.size()) op.arg = POST_PLAIN;
      if (zero_start && c == 0 && k == 0) op.arg = rf ? PRE_RESID : PRE_ZERO;
      if (zero_start && c + 1 == inner && k + 1 == G.prog.size() && op.arg == POST_MIXED) op.arg = POST_MIXED_KEEP;
      if ((e = run_op<float>(h, G, op, G.dL32, G.dP32, (float)relax(h), st)) != hipSuccess) return e;
      // the test of the iterate this pre-pass formed the residual of
      if (rf && c == 0 && k == 0 &&
          (e = launch_norm_finish<double>(G.dL64, G.gpre[0].ntx * G.gpre[0].nty, NORM_LAG, G.ns, st)) != hipSuccess)
        return e;
    }
  if (!G.mixed_fused && (e = launch_outer_update(G.dL64, G.dL32, G.shp[0], G.ns, st)) != hipSuccess) return e;
  if (rf) return hipSuccess;
  return launch_resnorm<double>(G.dL64, G.shp[0], NORM_CHECK, nullptr, G.dL32, stencil_kind(h), h->oned, G.ns, st);
}

// ----------------------------------------------------------------------- merged batched schedule

// Groups, by chain: a group joins the first merge whose deepest chain ends
// with the group's level shapes (same shapes level by level from its finest
// down); groups that fit no merge, and merges of one group, run their own
// cycles.  At most 32 groups per merge (participant sets are bit masks).
void form_merges(mg_handle h) {
  h->merges.clear();
  h->standalone.clear();
  if (!h->batched || h->groups.size() < 2) {
    for (int g = 0; g < (int)h->groups.size(); ++g) h->standalone.push_back(g);
    return;
  }
  std::vector<int> order(h->groups.size());
  for (int g = 0; g < (int)order.size(); ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return h->groups[a].nlev > h->groups[b].nlev; });
  auto ends_with = [&](const Group& D, const Group& G) {
    if (G.nlev > D.nlev) return false;
    const int o = D.nlev - G.nlev;
    for (int k = 0; k < G.nlev; ++k) {
      const LevelShape &a = D.shp[o + k], &b = G.shp[k];
      if (a.nx != b.nx || a.ny != b.ny || a.py != b.py) return false;
    }
    return true;
  };
  for (int g : order) {
    bool placed = false;
    for (Merge& M : h->merges)
      if (M.groups.size() < 32 && ends_with(h->groups[M.groups[0]], h->groups[g])) {
        M.groups.push_back(g);
        M.off.push_back(M.nlev - h->groups[g].nlev);
        placed = true;
        break;
      }
    if (!placed) {
      Merge M;
      M.groups = {g};
      M.off = {0};
      M.nlev = h->groups[g].nlev;
      h->merges.push_back(M);
    }
  }
  std::vector<Merge> keep;
  for (Merge& M : h->merges) {
    if (M.groups.size() == 1)
      h->standalone.push_back(M.groups[0]);
    else
      keep.push_back(M);
  }
  h->merges.swap(keep);
}

// Table of the participants in `set` (bit k: group M.groups[k]) on deepest-
// chain level l: level-major (one descriptor each) or, for the coarse-level
// kernel, problem-major (the levels from l down to the coarsest each).
int merge_table(Merge& M, const std::vector<Group>& groups, uint32_t set, int l, bool pm) {
  const std::string key = std::to_string(set) + "|" + std::to_string(l) + "|" + (pm ? "p" : "l");
  auto it = M.tab_index.find(key);
  if (it != M.tab_index.end()) return it->second;
  MTab t;
  for (int k = 0; k < (int)M.groups.size(); ++k) {
    if (!((set >> k) & 1)) continue;
    const Group& G = groups[M.groups[k]];
    const int ll = l - M.off[k];
    for (int sl = 0; sl < G.ns; ++sl) {
      if (pm)
        for (int q = ll; q < G.nlev; ++q) t.mem.push_back({M.groups[k], sl, q});
      else
        t.mem.push_back({M.groups[k], sl, ll});
    }
  }
  M.tabs.push_back(t);
  M.tab_index[key] = (int)M.tabs.size() - 1;
  return (int)M.tabs.size() - 1;
}

int participants(const Merge& M, const std::vector<Group>& groups, uint32_t set) {
  int n = 0;
  for (int k = 0; k < (int)M.groups.size(); ++k)
    if ((set >> k) & 1) n += groups[M.groups[k]].ns;
  return n;
}

// Walks the recursive cycle on the deepest chain (as Gen::host does) with
// the set of participating groups; a group joins the first call on its
// finest level.  Sub-cycles become H_SUB ops with their own program.
struct MergeGen {
  mg_handle h;
  Merge& M;
  const Gen& gen;  // on the deepest group
  std::vector<std::vector<Abs>>& subs;
  std::vector<uint32_t> sub_set;

  uint32_t joiners(int l) const {
    uint32_t m = 0;
    for (int k = 0; k < (int)M.off.size(); ++k)
      if (M.off[k] == l) m |= 1u << k;
    return m;
  }
  void push(int type, int l, int arg, uint32_t set, int fine) {
    if (!set) return;
    MOp op;
    op.type = type;
    op.level = l;
    op.arg = arg;
    op.fine = fine;
    op.n = (int)set;  // the set for now; replaced by the participant count when the tables are built
    M.prog.push_back(op);
  }
  void walk(int l, int kind, uint32_t active, bool lead) {
    const uint32_t fine = active & joiners(l), inner = active & ~fine;
    if (gen.small(l) || l == M.nlev - 1) {
      // groups whose finest level lies below this one run their own cycle,
      // which this call's program contains, as a launch of their own
      if (lead)
        for (int t = l + 1; t < M.nlev; ++t) {
          const uint32_t js = joiners(t);
          if (!js) continue;
          std::vector<Abs> own;
          gen.expand(own, t, kind);
          subs.push_back(own);
          sub_set.push_back(js);
          push(H_SUB, t, (int)subs.size() - 1, js, 0);
          push(H_NORM, t, 0, js, 1);
        }
      std::vector<Abs> body;
      gen.expand(body, l, kind);
      if (!M.prog.empty() && M.prog.back().type == H_SUB && M.prog.back().level == l &&
          sub_set[M.prog.back().arg] == active) {
        std::vector<Abs>& prev = subs[M.prog.back().arg];  // F then V on the same level and set: one launch
        for (const Abs& a : body)
          if (!(a.type == H_COARSE && !prev.empty() && prev.back().type == H_COARSE)) prev.push_back(a);
      } else {
        subs.push_back(body);
        sub_set.push_back(active);
        push(H_SUB, l, (int)subs.size() - 1, active, 0);
      }
      push(H_NORM, l, 0, fine, 1);
      return;
    }
    const bool fused = h->opts.tile_mode != MG_TILES_PER_OP;
    if (fused) {
      push(H_PRE, l, 0, fine, 1);
      push(H_PRE, l, 0, inner, 0);
    } else {
      std::vector<Abs> tmp;
      gen.smooth(tmp, l, h->opts.nu_pre);
      for (const Abs& a : tmp) push(a.type, l, a.arg, active, 0);
      push(H_DR, l, 0, active, 0);
    }
    // groups join only the leading call on their finest level (their cycle)
    const uint32_t next = lead ? (active | joiners(l + 1)) : active;
    if (kind == MG_CYCLE_F) {
      walk(l + 1, MG_CYCLE_F, next, lead);
      walk(l + 1, MG_CYCLE_V, active, false);
    } else if (kind == MG_CYCLE_W) {
      walk(l + 1, MG_CYCLE_W, next, lead);
      walk(l + 1, MG_CYCLE_W, active, false);
    } else {
      walk(l + 1, MG_CYCLE_V, next, lead);
    }
    if (h->opts.adaptive_omega) push(H_OMEGA, l, fused ? 1 : 0, active, 0);
    if (fused) {
      push(H_POST, l, POST_PLAIN, fine, 1);
      push(H_POST, l, POST_PLAIN, inner, 0);
      push(H_NORM, l, 1, fine, 1);
      return;
    }
    push(H_PROLONG, l, h->opts.adaptive_omega ? 1 : 0, active, 0);
    std::vector<Abs> tmp;
    gen.smooth(tmp, l, h->opts.nu_post);
    for (const Abs& a : tmp) push(a.type, l, a.arg, active, 0);
    push(H_NORM, l, 0, fine, 1);
  }
};

template <typename T>
Level<T>* table_ptr(const MTab& t);
template <>
Level<double>* table_ptr<double>(const MTab& t) { return t.d64; }
template <>
Level<float>* table_ptr<float>(const MTab& t) { return t.d32; }

// Host copies of a table's descriptors, from the groups' current ones.
template <typename T>
std::vector<Level<T>> table_rows(mg_handle h, const MTab& t) {
  std::vector<Level<T>> rows(t.mem.size());
  for (size_t e = 0; e < t.mem.size(); ++e) {
    const Group& G = h->groups[t.mem[e][0]];
    if constexpr (std::is_same<T, double>::value)
      rows[e] = G.l64(t.mem[e][2], t.mem[e][1]);
    else
      rows[e] = G.L32[(size_t)t.mem[e][2] * G.ns + t.mem[e][1]];
  }
  return rows;
}

mg_status upload_merge_tables(mg_handle h) {
  for (Merge& M : h->merges)
    for (MTab& t : M.tabs) {
      const std::vector<Level<double>> r64 = table_rows<double>(h, t);
      HIPCHK(h, hipMemcpyAsync(t.d64, r64.data(), r64.size() * sizeof(Level<double>), hipMemcpyHostToDevice, h->stream));
      if (h->mixed()) {
        const std::vector<Level<float>> r32 = table_rows<float>(h, t);
        HIPCHK(h, hipMemcpyAsync(t.d32, r32.data(), r32.size() * sizeof(Level<float>), hipMemcpyHostToDevice, h->stream));
      }
    }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return MG_OK;
}

// The merged program of every merge: ops, descriptor tables, sub-programs
// (levels relative to the sub-cycle's top) and tile shapes.
mg_status build_merges(mg_handle h) {
  form_merges(h);
  for (Merge& M : h->merges) {
    const Group& D = h->groups[M.groups[0]];
    Gen gen{h, D, D.threshold};
    std::vector<std::vector<Abs>> subs;
    MergeGen mg{h, M, gen, subs, {}};
    M.prog.clear();
    mg.walk(0, h->opts.cycle, mg.joiners(0), true);
    // tables, participant counts, tile shapes
    std::vector<DOp> flat;
    for (MOp& op : M.prog) {
      const uint32_t set = (uint32_t)op.n;
      op.n = participants(M, h->groups, set);
      if (op.type == H_SUB) {
        op.tab = merge_table(M, h->groups, set, op.level, true);
        // the sub-program with levels counted from op.level
        const std::vector<Abs>& body = subs[op.arg];
        const int b = (int)flat.size();
        for (const Abs& a : body) {
          int t = OP_COLOR;
          switch (a.type) {
            case H_COLOR: t = OP_COLOR; break;
            case H_JACOBI: t = OP_JACOBI; break;
            case H_COPY: t = OP_COPY; break;
            case H_DR: t = OP_DR; break;
            case H_PROLONG: t = OP_PROLONG; break;
            case H_COARSE: t = OP_COARSE; break;
            case H_LINE: t = OP_LINE; break;
            case H_OMEGA: t = OP_OMEGA; break;
          }
          flat.push_back({t, a.level - op.level, a.arg, 0});
        }
        fold_sweeps(flat, (size_t)b, h->ncol);
        fold_transfers(flat, (size_t)b);
        std::vector<int> beg(op.n, b), cnt(op.n, (int)(flat.size() - b));
        std::vector<double*> chol;  // one per participant: the first entry of its levels
        for (int k = 0; k < (int)M.groups.size(); ++k)
          if ((set >> k) & 1)
            for (int sl = 0; sl < h->groups[M.groups[k]].ns; ++sl) chol.push_back(h->groups[M.groups[k]].cinv[sl]);
        HIPCHK(h, h->dalloc(&op.dbeg, beg.size() * sizeof(int)));
        HIPCHK(h, h->dalloc(&op.dcnt, cnt.size() * sizeof(int)));
        HIPCHK(h, h->dalloc(&op.dchol, chol.size() * sizeof(double*)));
        HIPCHK(h, hipMemcpyAsync(op.dbeg, beg.data(), beg.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(op.dcnt, cnt.data(), cnt.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(op.dchol, chol.data(), chol.size() * sizeof(double*), hipMemcpyHostToDevice,
                                 h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        continue;
      }
      op.tab = merge_table(M, h->groups, set, op.level, false);
      if (op.type == H_PRE || op.type == H_POST || op.type == H_DR || op.type == H_PROLONG || op.type == H_OMEGA)
        op.ctab = merge_table(M, h->groups, set, op.level + 1, false);
      if (op.type == H_PRE)
        op.g = choose_tile_for(h, D.shp[op.level], op.n, sweeps(h, h->opts.nu_pre) + 2, false);
      if (op.type == H_POST)
        op.g = choose_tile_for(h, D.shp[op.level], op.n,
                               sweeps(h, h->opts.nu_post) + (op.fine && !h->mixed() ? 1 : 0), true);
    }
    if (std::getenv("MG_DEBUG_SCHEDULE")) {
      static const char* names[] = {"COLOR", "JACOBI", "COPY", "DR", "PROLONG", "COARSE", "SUB", "PRE",
                                    "POST", "LINE", "OMEGA", "NORM"};
      std::fprintf(stderr, "merged schedule: %zu groups, deepest %dx%d, %d levels\n", M.groups.size(), D.shp[0].nx,
                   D.shp[0].ny, M.nlev);
      for (size_t k = 0; k < M.groups.size(); ++k)
        std::fprintf(stderr, "  group %d (%dx%d, %d slots) joins at level %d\n", M.groups[k],
                     h->groups[M.groups[k]].shp[0].nx, h->groups[M.groups[k]].shp[0].ny, h->groups[M.groups[k]].ns,
                     M.off[k]);
      for (const MOp& op : M.prog)
        std::fprintf(stderr, "  %-7s level %d arg %d fine %d n %d tab %d ctab %d tile %d,%d,%d H %d\n",
                     names[op.type], op.level, op.arg, op.fine, op.n, op.tab, op.ctab, op.g.wide, op.g.TX, op.g.TY,
                     op.g.H);
    }
    if (!flat.empty()) {
      HIPCHK(h, h->dalloc(&M.dprog, flat.size() * sizeof(DOp)));
      HIPCHK(h, hipMemcpyAsync(M.dprog, flat.data(), flat.size() * sizeof(DOp), hipMemcpyHostToDevice, h->stream));
    }
    for (MTab& t : M.tabs) {
      HIPCHK(h, h->dalloc(&t.d64, t.mem.size() * sizeof(Level<double>)));
      if (h->mixed()) HIPCHK(h, h->dalloc(&t.d32, t.mem.size() * sizeof(Level<float>)));
    }
  }
  return upload_merge_tables(h);
}

// One merged op (inner: the FP32 cycle's number within a mixed outer step).
template <typename T>
hipError_t run_mop(mg_handle h, const Merge& M, const MOp& op, T omega, bool last_inner, hipStream_t st) {
  const Group& D = h->groups[M.groups[0]];
  const LevelShape& s = D.shp[op.level];
  Level<T>* Ls = table_ptr<T>(M.tabs[op.tab]);
  Level<T>* Cs = op.ctab >= 0 ? table_ptr<T>(M.tabs[op.ctab]) : nullptr;
  const int kind = stencil_kind(h);
  switch (op.type) {
    case H_COLOR: return launch_colour<T>(Ls, s, op.arg, h->ncol, omega, op.n, st);
    case H_JACOBI: return launch_jacobi<T>(Ls, s, op.arg, omega, op.n, st);
    case H_COPY: return launch_copy<T>(Ls, s, op.n, st);
    case H_DR: return launch_dr<T>(Ls, Cs, D.shp[op.level + 1], op.n, st);
    case H_PROLONG: return launch_prolong<T>(Ls, Cs, s, op.arg, op.n, st);
    case H_OMEGA: return launch_energy<T>(Ls, Cs, s, op.arg, kind, op.n, st);
    case H_PRE:
      return launch_pre<T>(Ls, Cs, op.g, h->opts.nu_pre, h->ncol, omega, kind, h->oned, op.fine != 0, op.n, st);
    case H_POST: {
      int mode = POST_PLAIN;
      if (op.fine) mode = h->mixed() ? (last_inner ? POST_MIXED : POST_PLAIN) : POST_NORM;
      const Level<double>* X64 = op.fine ? M.tabs[op.tab].d64 : nullptr;
      return launch_post<T>(Ls, Cs, op.g, h->opts.nu_post, h->ncol, omega, mode, X64, kind, h->oned, op.fine != 0,
                            op.n, st);
    }
    case H_SUB: {
      const int nl = D.nlev - op.level;
      const size_t bytes = sub_footprint(h, D, op.level);
      if (bytes <= SUB_LDS_BUDGET)
        return launch_subcycle_lds<T>(Ls, nl, 0, M.dprog, op.dbeg, op.dcnt, op.dchol, D.ncu, omega, h->ncol,
                                      h->ncol == 0 ? 3 : 2, kind, h->oned, bytes, op.n, st);
      return launch_subcycle<T>(Ls, nl, M.dprog, op.dbeg, op.dcnt, op.dchol, D.ncu, omega, h->ncol, op.n, st);
    }
  }
  return hipErrorInvalidValue;
}

// One merged cycle plus the stopping tests of every participating problem.
hipError_t enqueue_merged(mg_handle h, const Merge& M, hipStream_t st) {
  hipError_t e = hipSuccess;
  const int kind = stencil_kind(h);
  auto norm = [&](const MOp& op, bool mixed) -> hipError_t {
    const LevelShape& s = h->groups[M.groups[0]].shp[op.level];
    const MTab& t = M.tabs[op.tab];
    if (!mixed) return op.arg ? hipSuccess : launch_resnorm<double>(t.d64, s, NORM_CHECK, nullptr, nullptr, kind,
                                                                     h->oned, op.n, st);
    hipError_t r = hipSuccess;
    if (!op.arg && (r = launch_outer_update(t.d64, t.d32, s, op.n, st)) != hipSuccess) return r;
    return launch_resnorm<double>(t.d64, s, NORM_CHECK, nullptr, t.d32, kind, h->oned, op.n, st);
  };
  if (!h->mixed()) {
    for (const MOp& op : M.prog) {
      e = op.type == H_NORM ? norm(op, false) : run_mop<double>(h, M, op, relax(h), true, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int inner = inner_cycles(h);
  for (int c = 0; c < inner; ++c)
    for (const MOp& op : M.prog) {
      const bool last = c + 1 == inner;
      if (op.type == H_NORM) {
        if (last && (e = norm(op, true)) != hipSuccess) return e;
        continue;
      }
      if ((e = run_mop<float>(h, M, op, (float)relax(h), last, st)) != hipSuccess) return e;
    }
  return hipSuccess;
}

// Captures one cycle and eight cycles as graphs on a private stream (a graph
// can then be launched on any stream, the null stream included).  The groups
// of a batched handle become parallel branches (fork/join through events).
// Destroys the cycle graphs and their capture streams and events.
void drop_graphs(mg_handle h) {
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->g1) (void)hipGraphExecDestroy(h->g1);
  if (h->g8) (void)hipGraphExecDestroy(h->g8);
  h->g1 = h->g8 = nullptr;
  for (Group& G : h->groups) {
    if (G.branch && G.branch != h->cap) (void)hipStreamDestroy(G.branch);
    G.branch = nullptr;
  }
  for (Merge& M : h->merges) {
    if (M.branch && M.branch != h->cap) (void)hipStreamDestroy(M.branch);
    M.branch = nullptr;
  }
  if (h->cap) (void)hipStreamDestroy(h->cap);
  h->cap = nullptr;
  for (auto& ev : h->fork)
    if (ev) (void)hipEventDestroy(ev);
  h->fork.clear();
}

mg_status build_graphs(mg_handle h) {
  HIPCHK(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  // units: merged schedules, then groups that run their own cycle
  const int nm = (int)h->merges.size();
  const int nu = nm + (int)h->standalone.size();
  auto branch = [&](int u) -> hipStream_t& {
    return u < nm ? h->merges[u].branch : h->groups[h->standalone[u - nm]].branch;
  };
  auto enqueue = [&](int u, hipStream_t st) {
    return u < nm ? enqueue_merged(h, h->merges[u], st) : enqueue_cycle(h, h->groups[h->standalone[u - nm]], st);
  };
  h->fork.assign(2 * nu, nullptr);
  for (auto& ev : h->fork) HIPCHK(h, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  for (int u = 1; u < nu; ++u) HIPCHK(h, hipStreamCreateWithFlags(&branch(u), hipStreamNonBlocking));
  branch(0) = h->cap;
  for (int k : {1, 8}) {
    hipGraph_t graph = nullptr;
    HIPCHK(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int c = 0; c < k && e == hipSuccess; ++c) {
      if (nu == 1) {
        e = enqueue(0, h->cap);
        continue;
      }
      e = hipEventRecord(h->fork[0], h->cap);
      for (int u = 1; u < nu && e == hipSuccess; ++u) e = hipStreamWaitEvent(branch(u), h->fork[0], 0);
      for (int u = 0; u < nu && e == hipSuccess; ++u) e = enqueue(u, branch(u));
      for (int u = 1; u < nu && e == hipSuccess; ++u) {
        e = hipEventRecord(h->fork[nu + u], branch(u));
        if (e == hipSuccess) e = hipStreamWaitEvent(h->cap, h->fork[nu + u], 0);
      }
    }
    hipError_t e2 = hipStreamEndCapture(h->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(h, MG_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    if (k == 1) {
      size_t nodes = 0;
      if (hipGraphGetNodes(graph, nullptr, &nodes) == hipSuccess) h->graph_nodes = (int)nodes;
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
  if (g->nx < 3) return fail(nullptr, MG_EINVAL, "nx must be >= 3");
  if (g->periodic_y) {
    if (g->ny < 4 || (g->ny & 1)) return fail(nullptr, MG_EINVAL, "periodic ny must be even and >= 4");
  } else if (g->ny < 3) {
    return fail(nullptr, MG_EINVAL, "ny must be >= 3");
  }
  if ((long)g->nx * g->ny > (1L << 31) / 2) return fail(nullptr, MG_EINVAL, "grid too large");
  if (g->ys && g->periodic_y)
    return fail(nullptr, MG_EUNSUPPORTED, "refined y coordinates need a Dirichlet y direction");
  for (int d = 0; d < 2; ++d) {
    const double* c = d == 0 ? g->xs : g->ys;
    if (!c) continue;
    const int n = d == 0 ? g->nx : g->ny;
    const double len = d == 0 ? g->lx : g->ly;
    for (int k = 0; k < n; ++k)
      if (!std::isfinite(c[k]) || (k > 0 && !(c[k] > c[k - 1])))
        return fail(nullptr, MG_EINVAL, "node coordinates must be finite and strictly increasing");
    if (!(std::fabs(c[n - 1] - c[0] - len) <= 1e-12 * len))
      return fail(nullptr, MG_EINVAL, "node coordinates must span the domain length (lx or ly)");
  }
  return MG_OK;
}

// Line smoothers: the directions whose lines a smoothing step sweeps (bit 0
// x, bit 1 y; x first) and whether the lines are relaxed by Jacobi (TRI, ADI)
// or Gauss-Seidel (GSTRI, GSADI).
int line_dirs(int smoother) {
  switch (smoother) {
    case MG_SMOOTH_TRI_X:
    case MG_SMOOTH_GSTRI_X: return 1;
    case MG_SMOOTH_TRI_Y:
    case MG_SMOOTH_GSTRI_Y: return 2;
    case MG_SMOOTH_ADI:
    case MG_SMOOTH_GSADI: return 3;
    default: return 0;
  }
}
bool line_jacobi(int smoother) {
  return smoother == MG_SMOOTH_TRI_X || smoother == MG_SMOOTH_TRI_Y || smoother == MG_SMOOTH_ADI;
}

mg_status check_opts(const mg_options* o, int kind) {
  if (!o) return fail(nullptr, MG_EINVAL, "options is NULL");
  if (o->cycle != MG_CYCLE_F && o->cycle != MG_CYCLE_V && o->cycle != MG_CYCLE_W)
    return fail(nullptr, MG_EINVAL, "cycle must be F, V or W");
  if (o->smoother < MG_SMOOTH_JACOBI || o->smoother > MG_SMOOTH_GSADI) return fail(nullptr, MG_EINVAL, "bad smoother");
  if (o->smoother == MG_SMOOTH_RBGS && kind == MG_COEF_CELL9)
    return fail(nullptr, MG_EUNSUPPORTED, "red-black ordering does not decouple the 9-point stencil; use GS4C");
  if (o->nu_pre < 0 || o->nu_pre > 8 || o->nu_post < 0 || o->nu_post > 8)
    return fail(nullptr, MG_EINVAL, "nu_pre and nu_post must be in [0, 8]");
  if ((o->smoother == MG_SMOOTH_JACOBI || line_jacobi(o->smoother)) && !finite_pos(o->omega))
    return fail(nullptr, MG_EINVAL, "omega must be > 0");
  if (!(o->sor == 0.0 || (o->sor > 0.0 && o->sor < 2.0)))
    return fail(nullptr, MG_EINVAL, "sor must be in (0, 2), or 0 for plain Gauss-Seidel");
  if (o->precision != MG_PREC_FP64 && o->precision != MG_PREC_MIXED) return fail(nullptr, MG_EINVAL, "bad precision");
  if (o->coarse_cta_nodes < 0) return fail(nullptr, MG_EINVAL, "coarse_cta_nodes must be >= 0");
  if (o->tile_mode < MG_TILES_FUSED || o->tile_mode > MG_TILES_WIDE) return fail(nullptr, MG_EINVAL, "bad tile_mode");
  if (o->tile_x < 0 || o->tile_y < 0 || (o->tile_x & 1) || (o->tile_y & 1) || o->tile_x > 512 || o->tile_y > 512)
    return fail(nullptr, MG_EINVAL, "tile_x and tile_y must be even, in [0, 512]");
  if (o->inner_cycles < 0 || o->inner_cycles > 16) return fail(nullptr, MG_EINVAL, "inner_cycles must be in [0, 16]");
  if (o->coarse_op != MG_COARSE_DEFAULT && o->coarse_op != MG_COARSE_GALERKIN)
    return fail(nullptr, MG_EINVAL, "coarse_op must be MG_COARSE_DEFAULT or MG_COARSE_GALERKIN");
  if (o->adaptive_omega != 0 && o->adaptive_omega != 1) return fail(nullptr, MG_EINVAL, "adaptive_omega must be 0 or 1");
  if (o->tune < MG_TUNE_AUTO || o->tune > MG_TUNE_REFRESH) return fail(nullptr, MG_EINVAL, "bad tune mode");
  if (o->coarse_op == MG_COARSE_GALERKIN && kind == MG_COEF_CONST5 && o->smoother != MG_SMOOTH_JACOBI &&
      o->smoother != MG_SMOOTH_GS4C)
    return fail(nullptr, MG_EUNSUPPORTED,
                "Galerkin coarse levels of a 5-point problem are 9-point: use the Jacobi or four-colour smoother");
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
  drop_graphs(h);
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  h->ev0 = h->ev1 = nullptr;
}

int max_levels(int nx, int ny, int py) {
  int m = 1;
  while (can_coarsen(nx, ny, py)) {
    nx = (nx - 1) / 2 + 1;
    ny = py ? ny / 2 : (ny - 1) / 2 + 1;
    ++m;
  }
  return m;
}

// Shapes, buffers, operators, coarsest factors and descriptors of a group.
// Problem p = G.probs[s] uses h->eps_x[p], h->eps_y[p] (5-point) or the
// coefficient arrays in coeffs (9-point, single-problem handles only).
// Line-smoother storage of one level (factors for each swept direction and
// the forward-sweep scratch, all [ny][pitch]) and its factors.
template <typename T>
hipError_t alloc_line_factors(mg_handle h, Level<T>& L, const LevelShape& sh) {
  const size_t n = (size_t)L.pitch * sh.ny;
  hipError_t e = hipSuccess;
  for (int dir = 0; dir < 2; ++dir) {
    if (!((h->line >> dir) & 1)) continue;
    if ((e = h->dalloc(&L.lcp[dir], n * sizeof(T))) != hipSuccess) return e;
    if ((e = h->dalloc(&L.lid[dir], n * sizeof(T))) != hipSuccess) return e;
  }
  return h->dalloc(&L.lr, n * sizeof(T));
}

// Thomas factors of every line of every level (after the operators).
hipError_t assemble_line_factors(mg_handle h, Group& G) {
  hipError_t e = hipSuccess;
  for (int s = 0; s < G.ns; ++s)
    for (int l = 0; l < G.nlev; ++l)
      for (int dir = 0; dir < 2; ++dir) {
        if (!((h->line >> dir) & 1)) continue;
        e = h->mixed() ? launch_line_factor<float>(G.l32(l, s), dir, h->stream)
                       : launch_line_factor<double>(G.l64(l, s), dir, h->stream);
        if (e != hipSuccess) return e;
      }
  return hipSuccess;
}

// Operators of a cell-coefficient problem in the buffers setup_group
// allocated: finest bands from kx, ky, Galerkin bands of the coarser levels,
// inverse diagonals, the FP32 copies of a mixed hierarchy and the finest
// level's cell copies.  Queued on the handle's stream.
hipError_t assemble_cell9(mg_handle h, Group& G, const mg_coeffs* coeffs) {
  const mg_grid& grid = G.grid;
  const int ncx = grid.nx - 1;
  hipError_t e = hipSuccess;
  for (int l = 0; l < G.nlev; ++l) {
    const LevelShape& sh = G.shp[l];
    const Level<double>& L = G.l64(l, 0);
    const int brows = h->oned ? 1 : sh.ny;
    if (l == 0) {
      e = launch_q1_bands(G.band64[0], L.bstride, L.bpitch, brows, sh.nx, sh.ny, sh.py, coeffs->kx, coeffs->ky,
                          h->oned ? 0 : ncx, G.hx[0], G.hy[0], h->stream);
    } else {
      const LevelShape& f = G.shp[l - 1];
      const Level<double>& Lf = G.l64(l - 1, 0);
      e = launch_rap(G.band64[l], L.bstride, L.bpitch, brows, sh.nx, sh.ny, G.band64[l - 1], Lf.bstride, Lf.bpitch,
                     f.nx, f.ny, sh.py, h->stream);
    }
    if (e != hipSuccess) return e;
    if ((e = launch_inv_diag(G.band64[l], L.bstride, h->stream)) != hipSuccess) return e;
    if (h->mixed() && (e = launch_to_float(G.band64[l], G.band32[l], (long)NBANDS * L.bstride, h->stream)) != hipSuccess)
      return e;
  }
  const Level<double>& L0 = G.l64(0, 0);
  if (L0.kcx) {
    const LevelShape& sh = G.shp[0];
    const size_t nc = (size_t)ncx * (sh.py ? sh.ny : sh.ny - 1);
    const bool two = L0.kcy != L0.kcx;
    e = hipMemcpyAsync((void*)L0.kcx, coeffs->kx, nc * sizeof(double), hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess && two)
      e = hipMemcpyAsync((void*)L0.kcy, coeffs->ky, nc * sizeof(double), hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return e;
    if (h->mixed()) {
      const Level<float>& M = G.l32(0, 0);
      if ((e = launch_to_float(L0.kcx, (float*)M.kcx, (long)nc, h->stream)) != hipSuccess) return e;
      if (two && (e = launch_to_float(L0.kcy, (float*)M.kcy, (long)nc, h->stream)) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// Operators of a 5-point problem with Galerkin coarse levels, in the band
// buffers setup_group allocated: the finest level's 5-point couplings as 1-D
// bands (C = 2 (cx + cy), E = -cx, N = -cy, no corner couplings), the coarser
// levels' R A P, inverse diagonals and the FP32 copies of a mixed hierarchy.
hipError_t assemble_galerkin5(mg_handle h, Group& G) {
  const double cx = h->eps_x[0] / (G.hx[0] * G.hx[0]);
  const double cy = h->eps_y[0] / (G.hy[0] * G.hy[0]);
  const Level<double>& L0 = G.l64(0, 0);
  std::vector<double> fine((size_t)NBANDS * L0.bstride, 0.0);
  for (int i = 0; i < L0.bstride; ++i) {
    fine[i] = 2.0 * (cx + cy);
    fine[(size_t)L0.bstride + i] = -cx;
    fine[2 * (size_t)L0.bstride + i] = -cy;
  }
  hipError_t e = hipMemcpyAsync(G.band64[0], fine.data(), fine.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
  for (int l = 0; l < G.nlev && e == hipSuccess; ++l) {
    const LevelShape& sh = G.shp[l];
    const Level<double>& L = G.l64(l, 0);
    if (l > 0) {
      const LevelShape& f = G.shp[l - 1];
      const Level<double>& Lf = G.l64(l - 1, 0);
      e = launch_rap(G.band64[l], L.bstride, L.bpitch, 1, sh.nx, sh.ny, G.band64[l - 1], Lf.bstride, Lf.bpitch, f.nx,
                     f.ny, sh.py, h->stream);
    }
    if (e == hipSuccess) e = launch_inv_diag(G.band64[l], L.bstride, h->stream);
    if (e == hipSuccess && h->mixed())
      e = launch_to_float(G.band64[l], G.band32[l], (long)NBANDS * L.bstride, h->stream);
  }
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(h->stream);  // the host copy of the finest bands is about to go
}

// Dense coarsest operator of each slot, its Cholesky factor and the inverse
// the coarse solve applies, in the buffers setup_group allocated; waits for
// them and fails when an operator is not positive definite.
mg_status assemble_coarsest(mg_handle h, Group& G) {
  const int n = G.ncu;
  const LevelShape& sc = G.shp.back();
  for (int s = 0; s < G.ns; ++s) {
    const Level<double>& L = G.l64(G.nlev - 1, s);
    // the dense matrix is accumulated into a cleared buffer (it holds the
    // previous factor after an earlier assembly)
    HIPCHK(h, hipMemsetAsync(G.chol[s], 0, (size_t)n * n * sizeof(double), h->stream));
    HIPCHK(h, launch_dense_coarse(G.chol[s], n, sc.nx, sc.ny, sc.py, L.kind, L.cx, L.cy, L.dg, L.band, L.bstride,
                                  L.bpitch, h->stream));
    HIPCHK(h, launch_cholesky(G.chol[s], n, G.dinfo + s, h->stream));
    HIPCHK(h, launch_chol_inverse(G.chol[s], G.cinv[s], n, h->stream));
  }
  std::vector<int> info(G.ns, 0);
  HIPCHK(h, hipMemcpyAsync(info.data(), G.dinfo, (size_t)G.ns * sizeof(int), hipMemcpyDeviceToHost, h->stream));
  mg_status st = sync_check(h);
  if (st != MG_OK) return st;
  for (int s = 0; s < G.ns; ++s)
    if (info[s]) return fail(h, MG_EINVAL, "coarsest operator is not positive definite");
  return MG_OK;
}

mg_status setup_group(mg_handle h, Group& G, const mg_coeffs* coeffs, int32_t levels) {
  const mg_grid& grid = G.grid;
  const int py = grid.periodic_y ? 1 : 0;
  const int maxlev = max_levels(grid.nx, grid.ny, py);
  if (levels < 0 || levels > maxlev)
    return fail(h, MG_EINVAL, "grid " + std::to_string(grid.nx) + "x" + std::to_string(grid.ny) +
                                  " supports at most " + std::to_string(maxlev) + " levels");
  G.nlev = levels ? levels : maxlev;
  G.threshold = h->opts.coarse_cta_nodes;
  if (G.nlev > MAX_LEVELS) return fail(h, MG_EUNSUPPORTED, "more than " + std::to_string(MAX_LEVELS) + " levels");
  int nx = grid.nx, ny = grid.ny;
  for (int l = 0; l < G.nlev; ++l) {
    G.shp.push_back({nx, ny, py, py ? ny : ny - 2});
    G.hx.push_back(grid.lx / (nx - 1));
    G.hy.push_back(py ? grid.ly / ny : grid.ly / (ny - 1));
    nx = (nx - 1) / 2 + 1;
    ny = py ? ny / 2 : (ny - 1) / 2 + 1;
  }
  const LevelShape sc = G.shp.back();
  G.ncu = (sc.nx - 2) * sc.nrows;
  if (G.ncu > MAX_COARSE_UNKNOWNS)
    return fail(h, MG_EUNSUPPORTED, "coarsest grid has " + std::to_string(G.ncu) + " unknowns (max " +
                                        std::to_string(MAX_COARSE_UNKNOWNS) + "); use a grid that coarsens further");
  const int ns = G.ns;
  const bool mixed = h->mixed();

  // level buffers
  G.L64.assign((size_t)G.nlev * ns, Level<double>{});
  G.L32.assign(mixed ? (size_t)G.nlev * ns : 0, Level<float>{});
  for (int s = 0; s < ns; ++s) {
    SolveState* st = h->dstate + G.probs[s];
    for (int l = 0; l < G.nlev; ++l) {
      const LevelShape& sh = G.shp[l];
      if (l == 0) {
        // finest FP64 level: x and b are the caller's arrays (pitch nx)
        G.l64(0, s) = make_level<double>(sh, sh.nx, st);
        if (!mixed) HIPCHK(h, h->dalloc(&G.l64(0, s).t, (size_t)sh.nx * sh.ny * sizeof(double)));
      } else {
        const int p = round_up(sh.nx, 16);
        Level<double>& L = G.l64(l, s);
        L = make_level<double>(sh, p, st);
        if (!mixed) {
          HIPCHK(h, h->dalloc(&L.x, (size_t)p * sh.ny * sizeof(double)));
          HIPCHK(h, h->dalloc(&L.b, (size_t)p * sh.ny * sizeof(double)));
          HIPCHK(h, h->dalloc(&L.t, (size_t)p * sh.ny * sizeof(double)));
        }
      }
      if (mixed) {
        const int p = round_up(sh.nx, 32);
        Level<float>& L = G.l32(l, s);
        L = make_level<float>(sh, p, st);
        HIPCHK(h, h->dalloc(&L.x, (size_t)p * sh.ny * sizeof(float)));
        HIPCHK(h, h->dalloc(&L.b, (size_t)p * sh.ny * sizeof(float)));
        HIPCHK(h, h->dalloc(&L.t, (size_t)p * sh.ny * sizeof(float)));
      }
    }
  }
  // adaptive omega_l: one device scalar per (level, slot) below the
  // coarsest, in the precision of the cycle, starting at 1
  if (h->opts.adaptive_omega) {
    const size_t nw = (size_t)G.nlev * ns;
    if (mixed) {
      float* w = nullptr;
      HIPCHK(h, h->dalloc(&w, nw * sizeof(float)));
      const std::vector<float> ones(nw, 1.0f);
      HIPCHK(h, hipMemcpyAsync(w, ones.data(), nw * sizeof(float), hipMemcpyHostToDevice, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      for (int s = 0; s < ns; ++s)
        for (int l = 0; l + 1 < G.nlev; ++l) G.l32(l, s).wl = w + (size_t)l * ns + s;
    } else {
      double* w = nullptr;
      HIPCHK(h, h->dalloc(&w, nw * sizeof(double)));
      const std::vector<double> ones(nw, 1.0);
      HIPCHK(h, hipMemcpyAsync(w, ones.data(), nw * sizeof(double), hipMemcpyHostToDevice, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      for (int s = 0; s < ns; ++s)
        for (int l = 0; l + 1 < G.nlev; ++l) G.l64(l, s).wl = w + (size_t)l * ns + s;
    }
  }

  // operators
  if (stencil_kind(h) == ST5) {
    for (int s = 0; s < ns; ++s) {
      const int p = G.probs[s];
      for (int l = 0; l < G.nlev; ++l) {
        const double cx = h->eps_x[p] / (G.hx[l] * G.hx[l]);
        const double cy = h->eps_y[p] / (G.hy[l] * G.hy[l]);
        const double dg = 2.0 * (cx + cy);
        Level<double>& L = G.l64(l, s);
        L.kind = ST5;
        L.cx = cx;
        L.cy = cy;
        L.dg = dg;
        L.inv_dg = 1.0 / dg;
        if (mixed) {
          Level<float>& M = G.l32(l, s);
          M.kind = ST5;
          M.cx = (float)cx;
          M.cy = (float)cy;
          M.dg = (float)dg;
          M.inv_dg = (float)(1.0 / dg);
        }
      }
    }
  } else {
    // bands of every level, the finest level's cell copies (filled by
    // assemble_cell9)
    const int ncx = grid.nx - 1;
    G.band64.resize(G.nlev);
    G.band32.resize(G.nlev);
    for (int l = 0; l < G.nlev; ++l) {
      const LevelShape& sh = G.shp[l];
      const int bp = round_up(sh.nx, 16);
      const int bstride = bp * (h->oned ? 1 : sh.ny);
      HIPCHK(h, h->dalloc(&G.band64[l], (size_t)NBANDS * bstride * sizeof(double)));
      Level<double>& L = G.l64(l, 0);
      L.kind = ST9;
      L.band = G.band64[l];
      L.bpitch = h->oned ? 0 : bp;
      L.bstride = bstride;
      if (mixed) {
        HIPCHK(h, h->dalloc(&G.band32[l], (size_t)NBANDS * bstride * sizeof(float)));
        Level<float>& M = G.l32(l, 0);
        M.kind = ST9;
        M.band = G.band32[l];
        M.bpitch = L.bpitch;
        M.bstride = bstride;
      }
    }
    // finest level, coefficients varying in both directions, not run by the
    // coarse-level interpreter: own copies of the per-cell kx, ky, from which
    // the kernels of that level form its couplings (one copy when the caller
    // passes the same array for both)
    if (!h->oned && !Gen{h, G, G.threshold}.small(0)) {
      const LevelShape& sh = G.shp[0];
      const size_t nc = (size_t)ncx * (sh.py ? sh.ny : sh.ny - 1);
      const bool same = coeffs->kx == coeffs->ky;
      Level<double>& L = G.l64(0, 0);
      double* kc[2] = {nullptr, nullptr};
      for (int d = 0; d < (same ? 1 : 2); ++d) HIPCHK(h, h->dalloc(&kc[d], nc * sizeof(double)));
      if (same) kc[1] = kc[0];
      const double ax = 1.0 / (G.hx[0] * G.hx[0]), ay = 1.0 / (G.hy[0] * G.hy[0]);
      L.kcx = kc[0];
      L.kcy = kc[1];
      L.kcpitch = ncx;
      L.kc3x = ax / 3.0;
      L.kc3y = ay / 3.0;
      L.kc6x = ax / 6.0;
      L.kc6y = ay / 6.0;
      if (mixed) {
        float* kf[2] = {nullptr, nullptr};
        for (int d = 0; d < (same ? 1 : 2); ++d) HIPCHK(h, h->dalloc(&kf[d], nc * sizeof(float)));
        if (same) kf[1] = kf[0];
        Level<float>& M = G.l32(0, 0);
        M.kcx = kf[0];
        M.kcy = kf[1];
        M.kcpitch = ncx;
        M.kc3x = (float)L.kc3x;
        M.kc3y = (float)L.kc3y;
        M.kc6x = (float)L.kc6x;
        M.kc6y = (float)L.kc6y;
      }
    }
    HIPCHK(h, h->galerkin5 ? assemble_galerkin5(h, G) : assemble_cell9(h, G, coeffs));
  }

  // line smoothers: Thomas factors of every line of the cycle's hierarchy
  if (h->line) {
    for (int s = 0; s < ns; ++s)
      for (int l = 0; l < G.nlev; ++l) {
        const LevelShape& sh = G.shp[l];
        if (mixed) {
          HIPCHK(h, alloc_line_factors(h, G.l32(l, s), sh));
        } else {
          HIPCHK(h, alloc_line_factors(h, G.l64(l, s), sh));
        }
      }
    HIPCHK(h, assemble_line_factors(h, G));
  }

  // coarsest operator of each slot: dense matrix, Cholesky factor and the
  // inverse the coarse solve applies (FP64)
  {
    const int n = G.ncu;
    G.chol.assign(ns, nullptr);
    G.cinv.assign(ns, nullptr);
    HIPCHK(h, h->dalloc(&G.dinfo, (size_t)ns * sizeof(int)));
    for (int s = 0; s < ns; ++s) {
      HIPCHK(h, h->dalloc(&G.chol[s], (size_t)n * n * sizeof(double)));
      HIPCHK(h, h->dalloc(&G.cinv[s], (size_t)n * n * sizeof(double)));
    }
    HIPCHK(h, h->dalloc(&G.dcholp, (size_t)ns * sizeof(double*)));
    HIPCHK(h, hipMemcpyAsync(G.dcholp, G.cinv.data(), (size_t)ns * sizeof(double*), hipMemcpyHostToDevice,
                             h->stream));
    mg_status st = assemble_coarsest(h, G);
    if (st != MG_OK) return st;
  }

  // descriptors: level-major and problem-major copies
  const size_t nd = (size_t)G.nlev * ns;
  HIPCHK(h, h->dalloc(&G.dL64, nd * sizeof(Level<double>)));
  HIPCHK(h, h->dalloc(&G.dP64, nd * sizeof(Level<double>)));
  if (mixed) {
    HIPCHK(h, h->dalloc(&G.dL32, nd * sizeof(Level<float>)));
    HIPCHK(h, h->dalloc(&G.dP32, nd * sizeof(Level<float>)));
  }
  return build_program(h, G);
}

// Uploads both descriptor layouts of a group (after the finest level's caller
// arrays changed) and waits for the copies.
mg_status upload_descriptors(mg_handle h, Group& G) {
  const size_t nd = (size_t)G.nlev * G.ns;
  hipStream_t st = h->stream;
  std::vector<Level<double>> p64(nd);
  for (int s = 0; s < G.ns; ++s)
    for (int l = 0; l < G.nlev; ++l) p64[(size_t)s * G.nlev + l] = G.l64(l, s);
  HIPCHK(h, hipMemcpyAsync(G.dL64, G.L64.data(), nd * sizeof(Level<double>), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(G.dP64, p64.data(), nd * sizeof(Level<double>), hipMemcpyHostToDevice, st));
  std::vector<Level<float>> p32;
  if (h->mixed()) {
    p32.resize(nd);
    for (int s = 0; s < G.ns; ++s)
      for (int l = 0; l < G.nlev; ++l) p32[(size_t)s * G.nlev + l] = G.l32(l, s);
    HIPCHK(h, hipMemcpyAsync(G.dL32, G.L32.data(), nd * sizeof(Level<float>), hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(G.dP32, p32.data(), nd * sizeof(Level<float>), hipMemcpyHostToDevice, st));
  }
  HIPCHK(h, hipStreamSynchronize(st));
  return MG_OK;
}

// Counts the cell coefficients that are not finite and > 0 (one read-only
// device pass over kx and ky) and fails if there are any.
mg_status check_cell_coeffs(mg_handle h, const mg_coeffs* coeffs) {
  const mg_grid& grid = h->groups[0].grid;
  const int ncx = grid.nx - 1, ncy = grid.periodic_y ? grid.ny : grid.ny - 1;
  const long nc = h->in_oned ? ncx : (long)ncx * ncy;
  HIPCHK(h, hipMemsetAsync(h->dcount, 0, sizeof(int), h->stream));
  HIPCHK(h, launch_count_bad(coeffs->kx, nc, h->dcount, h->stream));
  HIPCHK(h, launch_count_bad(coeffs->ky, nc, h->dcount, h->stream));
  int bad = 0;
  HIPCHK(h, hipMemcpyAsync(&bad, h->dcount, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  mg_status s = sync_check(h);
  if (s != MG_OK) return s;
  if (bad) return fail(h, MG_EINVAL, std::to_string(bad) + " coefficient values are not finite and > 0");
  return MG_OK;
}

// ----------------------------------------------------------------------- autotuner
//
// Results are bitwise independent of the tile shape of a fused pass and of
// the level from which the single-workgroup kernel takes over, so both are
// free to choose for speed.  For each threshold candidate (the default, one
// more fused level, one more interpreted level) the program is built, every
// fused pass is timed on the handle's own buffers for each candidate tile
// (wide tiles of several heights, small tiles of several shapes, and the
// fixed rule's choice) and the fastest is kept; then whole cycles decide the
// threshold.  Choices are cached (mg_tune.hip) under keys that carry the
// device architecture and the kernel-source digest.

bool tiles_fixed(mg_handle h) {
  return h->opts.tile_mode != MG_TILES_FUSED || h->opts.tile_x != 0 || h->opts.tile_y != 0;
}

std::string geom_str(const TileGeom& g) {
  return std::to_string(g.wide) + "," + std::to_string(g.TX) + "," + std::to_string(g.TY);
}

bool geom_parse(const std::string& v, const LevelShape& s, int H, int Hy, TileGeom& g) {
  int w = 0, tx = 0, ty = 0;
  if (std::sscanf(v.c_str(), "%d,%d,%d", &w, &tx, &ty) != 3 || tx < 2 || ty < 2) return false;
  g = w ? wide_geom(s.nx, s.ny, ty, H, Hy) : tile_geom(s.nx, s.ny, tx, ty, H);
  return !w || g.TX == tx;
}

std::string pass_key(mg_handle h, const Group& G, const HostOp& op, int H) {
  const LevelShape& s = G.shp[op.level];
  std::ostringstream k;
  k << "pass|" << tune_identity() << "|" << (h->mixed() ? "f32" : "f64") << "|st" << stencil_kind(h) << "|b1"
    << (stencil_kind(h) == ST9 && h->oned) << "|cells" << (G.l64(op.level, 0).kcx != nullptr) << "|col" << h->ncol
    << "|" << (op.type == H_PRE ? "pre" : "post") << op.arg << "|nu"
    << (op.type == H_PRE ? h->opts.nu_pre : h->opts.nu_post) << "|H" << H << "|sor" << (relax(h) != 1.0)
    << "|aw" << h->opts.adaptive_omega << "|" << s.nx << "x" << s.ny << "p" << s.py << "|z" << G.ns << "|fine"
    << (op.level == 0) << "|cu" << h->ncus;
  return k.str();
}

std::string threshold_key(mg_handle h, const Group& G) {
  std::ostringstream k;
  k << "coarse|" << tune_identity() << "|" << (h->mixed() ? "f32" : "f64") << "|st" << stencil_kind(h) << "|b1"
    << (stencil_kind(h) == ST9 && h->oned) << "|sm" << h->opts.smoother << "|nu" << h->opts.nu_pre << ","
    << h->opts.nu_post << "|cy" << h->opts.cycle << "|in" << inner_cycles(h) << "|aw" << h->opts.adaptive_omega
    << "|tm" << h->opts.tile_mode << "|" << G.shp[0].nx << "x" << G.shp[0].ny << "p" << G.shp[0].py << "|L"
    << G.nlev << "|z" << G.ns << "|cu" << h->ncus;
  return k.str();
}

// Candidate tiles of one fused pass (LDS within the fused-pass cap).
std::vector<TileGeom> tile_candidates(mg_handle h, const LevelShape& s, int ns, int H, bool post) {
  auto lds = [&](const TileGeom& g) {
    if (h->mixed()) return post ? post_lds_bytes<float>(g, h->ncol) : pre_lds_bytes<float>(g, h->ncol);
    return post ? post_lds_bytes<double>(g, h->ncol) : pre_lds_bytes<double>(g, h->ncol);
  };
  std::vector<TileGeom> out;
  out.push_back(choose_tile_for(h, s, ns, H, post));  // the fixed rule first
  if (2 * H < wide_width())
    for (int ty = 8; ty <= 128; ty += (ty < 64 ? 8 : 16)) {
      const TileGeom g = wide_geom(s.nx, s.ny, ty, H, row_halo(h, H, post));
      if (lds(g) <= FUSED_LDS_MAX && (long)g.ntx * g.nty * ns <= 64L * h->ncus) out.push_back(g);
    }
  for (int tx : {16, 32, 64, 128})
    for (int ty : {4, 8, 16, 32}) {
      const TileGeom g = tile_geom(s.nx, s.ny, tx, ty, H);
      if (lds(g) <= FUSED_LDS_MAX && (long)g.ntx * g.nty * ns <= 64L * h->ncus) out.push_back(g);
    }
  return out;
}

// Average device time (us) of `reps` runs of `ops` on the handle's stream
// after one untimed run.
template <typename T>
hipError_t time_ops(mg_handle h, Group& G, const std::vector<HostOp>& ops, Level<T>* dL, Level<T>* dP, T omega,
                    int reps, double* us) {
  hipStream_t st = h->stream;
  hipError_t e = hipSuccess;
  for (int r = 0; r <= reps; ++r) {
    if (r == 1 && (e = hipEventRecord(h->ev0, st)) != hipSuccess) return e;
    for (const HostOp& op : ops)
      if ((e = run_op<T>(h, G, op, dL, dP, omega, st)) != hipSuccess) return e;
  }
  if ((e = hipEventRecord(h->ev1, st)) != hipSuccess) return e;
  if ((e = hipEventSynchronize(h->ev1)) != hipSuccess) return e;
  float ms = 0.f;
  if ((e = hipEventElapsedTime(&ms, h->ev0, h->ev1)) != hipSuccess) return e;
  *us = 1e3 * ms / reps;
  return hipSuccess;
}

hipError_t time_pass(mg_handle h, Group& G, const HostOp& op, double* us) {
  const std::vector<HostOp> one{op};
  if (h->mixed()) return time_ops<float>(h, G, one, G.dL32, G.dP32, (float)relax(h), 3, us);
  return time_ops<double>(h, G, one, G.dL64, G.dP64, relax(h), 3, us);
}

hipError_t time_cycle(mg_handle h, Group& G, double* us) {
  hipStream_t st = h->stream;
  hipError_t e = hipSuccess;
  for (int r = 0; r <= 3; ++r) {
    if (r == 1 && (e = hipEventRecord(h->ev0, st)) != hipSuccess) return e;
    if ((e = enqueue_cycle(h, G, st)) != hipSuccess) return e;
  }
  if ((e = hipEventRecord(h->ev1, st)) != hipSuccess) return e;
  if ((e = hipEventSynchronize(h->ev1)) != hipSuccess) return e;
  float ms = 0.f;
  if ((e = hipEventElapsedTime(&ms, h->ev0, h->ev1)) != hipSuccess) return e;
  *us = 1e3 * ms / 3;
  return hipSuccess;
}

// Tile of every fused pass of the group's current program: cached, or the
// fastest candidate (the rule's choice unless another is 2 % faster).
mg_status tune_tiles(mg_handle h, Group& G) {
  const bool refresh = h->opts.tune == MG_TUNE_REFRESH;
  for (const HostOp& op : G.prog) {
    if (op.type != H_PRE && op.type != H_POST) continue;
    const bool post = op.type == H_POST;
    TileGeom& slot = post ? G.gpost[op.level] : G.gpre[op.level];
    const int H = slot.H;
    const std::string key = pass_key(h, G, op, H);
    TileGeom g{};
    const std::string v = refresh ? std::string() : tune_lookup(key);
    if (!v.empty() && geom_parse(v, G.shp[op.level], H, row_halo(h, H, post), g)) {
      slot = g;
      continue;
    }
    const std::vector<TileGeom> cands = tile_candidates(h, G.shp[op.level], G.ns, H, post);
    TileGeom best = cands[0];
    double best_us = 0.0;
    for (size_t c = 0; c < cands.size(); ++c) {
      slot = cands[c];
      double us = 0.0;
      HIPCHK(h, time_pass(h, G, op, &us));
      if (c == 0 || us < best_us * (best.TX == cands[0].TX && best.TY == cands[0].TY && best.wide == cands[0].wide
                                        ? 0.98 : 1.0)) {
        best = cands[c];
        best_us = us;
      }
    }
    slot = best;
    tune_store(key, geom_str(best));
  }
  return MG_OK;
}

// Tiles and coarse threshold of every group (setup, after the descriptors
// and partial-sum buffers exist).  The finest FP64 level borrows two
// scratch arrays for the caller's x and b; the stopping states are set so
// that no candidate run stops early, and reset by the next solve.
// Tiles of every fused op of a merged schedule (cached, or the fastest
// candidate for its level shape and number of participants).
mg_status tune_merge_tiles(mg_handle h, Merge& M) {
  const bool refresh = h->opts.tune == MG_TUNE_REFRESH;
  const Group& D = h->groups[M.groups[0]];
  for (MOp& op : M.prog) {
    if (op.type != H_PRE && op.type != H_POST) continue;
    const bool post = op.type == H_POST;
    const int H = op.g.H;
    const LevelShape& s = D.shp[op.level];
    std::ostringstream k;
    k << "mpass|" << tune_identity() << "|" << (h->mixed() ? "f32" : "f64") << "|st" << stencil_kind(h) << "|col"
      << h->ncol << "|" << (post ? "post" : "pre") << "|nu" << (post ? h->opts.nu_post : h->opts.nu_pre) << "|H" << H
      << "|sor" << (relax(h) != 1.0) << "|aw" << h->opts.adaptive_omega << "|" << s.nx << "x" << s.ny << "p" << s.py
      << "|z" << op.n << "|fine" << op.fine << "|cu" << h->ncus;
    const std::string key = k.str();
    TileGeom g{};
    const std::string v = refresh ? std::string() : tune_lookup(key);
    if (!v.empty() && geom_parse(v, s, H, row_halo(h, H, post), g)) {
      op.g = g;
      continue;
    }
    const std::vector<TileGeom> cands = tile_candidates(h, s, op.n, H, post);
    TileGeom best = cands[0];
    double best_us = 0.0;
    for (size_t c = 0; c < cands.size(); ++c) {
      op.g = cands[c];
      hipError_t e = hipSuccess;
      for (int r = 0; r <= 3 && e == hipSuccess; ++r) {
        if (r == 1) e = hipEventRecord(h->ev0, h->stream);
        if (e == hipSuccess)
          e = h->mixed() ? run_mop<float>(h, M, op, (float)relax(h), true, h->stream)
                         : run_mop<double>(h, M, op, relax(h), true, h->stream);
      }
      if (e == hipSuccess) e = hipEventRecord(h->ev1, h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(h->ev1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, h->ev0, h->ev1);
      if (e != hipSuccess) return fail(h, MG_EDEVICE, std::string("tuning: ") + hipGetErrorString(e));
      const double us = 1e3 * ms / 3;
      const bool rule = best.TX == cands[0].TX && best.TY == cands[0].TY && best.wide == cands[0].wide;
      if (c == 0 || us < best_us * (rule ? 0.98 : 1.0)) {
        best = cands[c];
        best_us = us;
      }
    }
    op.g = best;
    tune_store(key, geom_str(best));
  }
  return MG_OK;
}

// Threshold and tiles of a group that runs its own cycle.
mg_status tune_group(mg_handle h, Group& G, bool tile_free, bool thr_free) {
  // threshold candidates: the default, one more fused level, one more
  // level in the single-workgroup kernel (global memory)
  // (not with the adaptive omega_l: the single-workgroup kernel sums its
  // level-wide products in another order than the launched reduction, so
  // moving a level between them changes the weight's rounding)
  std::vector<int> ths{0};
  if (thr_free && h->groups.size() == 1 && !h->opts.adaptive_omega) {
    Gen g0{h, G, 0};
    int top = 0;
    while (top < G.nlev - 1 && !g0.small(top)) ++top;
    const long ntop = (long)G.shp[top].nx * G.shp[top].ny;
    if (top < G.nlev - 1) ths.push_back((int)(ntop - 1));
    // (not the finest level when it forms its couplings from cells: the
    // single-workgroup kernel reads bands, equal only up to rounding)
    if (top > 0 && !(top == 1 && G.l64(0, 0).kcx)) ths.push_back((int)((long)G.shp[top - 1].nx * G.shp[top - 1].ny));
    const std::string cached = h->opts.tune == MG_TUNE_REFRESH ? std::string() : tune_lookup(threshold_key(h, G));
    if (!cached.empty()) ths.assign(1, std::atoi(cached.c_str()));
  } else if (!thr_free) {
    ths.assign(1, h->opts.coarse_cta_nodes);
  }
  int best_th = ths[0];
  double best_us = 0.0;
  mg_status res = MG_OK;
  for (size_t c = 0; c < ths.size() && res == MG_OK; ++c) {
    G.threshold = ths[c];
    res = build_program(h, G);
    if (res == MG_OK && tile_free) res = tune_tiles(h, G);
    if (res != MG_OK || ths.size() == 1) break;
    double us = 0.0;
    hipError_t te = time_cycle(h, G, &us);
    if (te != hipSuccess) return fail(h, MG_EDEVICE, std::string("tuning: ") + hipGetErrorString(te));
    if (c == 0 || us < best_us * (best_th == ths[0] ? 0.98 : 1.0)) {
      best_th = ths[c];
      best_us = us;
    }
  }
  if (res == MG_OK && ths.size() > 1) {
    tune_store(threshold_key(h, G), std::to_string(best_th));
    G.threshold = best_th;
    res = build_program(h, G);
    if (res == MG_OK && tile_free) res = tune_tiles(h, G);  // cached by now
  }
  // mixed form: the finest pre-pass forming the residual itself, or the
  // residual kernel after each cycle (same iterates bit for bit): the
  // pre-pass then loads the FP64 x and b over its whole region, halo
  // included, so whether it pays depends on the tile (kept only when 1 %
  // faster).  Tiles given by the caller keep the in-pass residual.
  G.resid_kernel = false;
  if (res == MG_OK && tile_free && resid_possible(h, G)) {
    const std::string key = threshold_key(h, G) + "|resid|" + geom_str(G.gpre[0]);
    const std::string cached = h->opts.tune == MG_TUNE_REFRESH ? std::string() : tune_lookup(key);
    if (!cached.empty()) {
      G.resid_kernel = cached == "kernel";
    } else {
      double us[2] = {0.0, 0.0};
      for (int v = 0; v < 2; ++v) {
        G.resid_kernel = v == 1;
        hipError_t te = time_cycle(h, G, &us[v]);
        if (te != hipSuccess) return fail(h, MG_EDEVICE, std::string("tuning: ") + hipGetErrorString(te));
      }
      G.resid_kernel = !(us[0] < 0.99 * us[1]);
      tune_store(key, G.resid_kernel ? "kernel" : "pass");
    }
  }
  return res;
}

// Batched handles with merged schedules: time one-cycle graph replays of
// the merged layout and of every group on its own branch, keep the faster
// (both give the same iterates bit for bit).
mg_status tune_schedule(mg_handle h) {
  std::ostringstream k;
  k << "sched|" << tune_identity() << "|" << (h->mixed() ? "f32" : "f64") << "|sm" << h->opts.smoother << "|nu"
    << h->opts.nu_pre << "," << h->opts.nu_post << "|cy" << h->opts.cycle << "|in" << inner_cycles(h) << "|aw"
    << h->opts.adaptive_omega << "|tm" << h->opts.tile_mode << "|cu" << h->ncus;
  for (const Group& G : h->groups) k << "|" << G.shp[0].nx << "x" << G.shp[0].ny << "p" << G.shp[0].py << "L" << G.nlev << "z" << G.ns;
  const std::string key = k.str();
  std::string choice = h->opts.tune == MG_TUNE_REFRESH ? std::string() : tune_lookup(key);
  auto split = [&]() {  // every merged group back on a branch of its own
    for (const Merge& M : h->merges)
      for (int g : M.groups) h->standalone.push_back(g);
    h->merges.clear();
  };
  if (choice == "branches") {
    split();
    return MG_OK;
  }
  if (choice == "merged") return MG_OK;
  double t[2] = {0.0, 0.0};
  std::vector<Merge> saved = h->merges;
  std::vector<int> saved_alone = h->standalone;
  for (int v = 0; v < 2; ++v) {
    if (v == 1) split();
    mg_status s = build_graphs(h);
    if (s != MG_OK) return s;
    for (int r = 0; r <= 3; ++r) {
      if (r == 1) HIPCHK(h, hipEventRecord(h->ev0, h->stream));
      HIPCHK(h, hipGraphLaunch(h->g1, h->stream));
    }
    HIPCHK(h, hipEventRecord(h->ev1, h->stream));
    HIPCHK(h, hipEventSynchronize(h->ev1));
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
    t[v] = ms;
    drop_graphs(h);
  }
  const bool merged = t[0] <= t[1];
  if (merged) {
    h->merges = saved;
    h->standalone = saved_alone;
  }
  tune_store(key, merged ? "merged" : "branches");
  return MG_OK;
}

// Tiles and coarse threshold of every group and merged schedule (setup,
// after the descriptors and partial-sum buffers exist).  Each group's finest
// FP64 level borrows two scratch arrays for the caller's x and b; the
// stopping states are set so that no candidate run stops early, and reset by
// the next solve.
mg_status tune_handle(mg_handle h) {
  if (h->opts.tune == MG_TUNE_OFF) return MG_OK;
  const bool tile_free = !tiles_fixed(h);
  const bool thr_free = h->opts.coarse_cta_nodes == 0;
  if (!tile_free && !thr_free) return MG_OK;
  hipStream_t st = h->stream;
  std::vector<SolveState> run(h->nprob);
  for (int p = 0; p < h->nprob; ++p) {
    run[p] = SolveState{};
    run[p].r0 = 1e300;  // never converged (tol < 0), never diverged
    run[p].tol = -1.0;
    run[p].partial = h->dpartial[p];
  }
  HIPCHK(h, hipMemcpyAsync(h->dstate, run.data(), run.size() * sizeof(SolveState), hipMemcpyHostToDevice, st));
  std::vector<double*> scratch;
  mg_status res = MG_OK;
  for (Group& G : h->groups) {
    const size_t n0 = (size_t)G.shp[0].nx * G.shp[0].ny;
    double *tx = nullptr, *tb = nullptr;
    hipError_t e = hipMalloc(&tx, n0 * sizeof(double));
    if (e == hipSuccess) scratch.push_back(tx);
    if (e == hipSuccess) e = hipMalloc(&tb, n0 * sizeof(double));
    if (e == hipSuccess) scratch.push_back(tb);
    if (e == hipSuccess) e = hipMemsetAsync(tx, 0, n0 * sizeof(double), st);
    if (e == hipSuccess) e = hipMemsetAsync(tb, 0, n0 * sizeof(double), st);
    if (e != hipSuccess) {
      res = fail(h, e == hipErrorOutOfMemory ? MG_ENOMEM : MG_EDEVICE, std::string("tuning scratch: ") +
                                                                            hipGetErrorString(e));
      break;
    }
    for (int sl = 0; sl < G.ns; ++sl) {
      G.l64(0, sl).x = tx;
      G.l64(0, sl).b = tb;
    }
    res = upload_descriptors(h, G);
    if (res != MG_OK) break;
  }
  if (res == MG_OK && !h->merges.empty()) res = upload_merge_tables(h);
  for (size_t u = 0; u < h->standalone.size() && res == MG_OK; ++u)
    res = tune_group(h, h->groups[h->standalone[u]], tile_free, thr_free);
  for (size_t m = 0; m < h->merges.size() && res == MG_OK && tile_free; ++m) res = tune_merge_tiles(h, h->merges[m]);
  if (res == MG_OK && !h->merges.empty()) res = tune_schedule(h);
  (void)hipStreamSynchronize(st);
  for (double* q : scratch) (void)hipFree(q);
  for (Group& G : h->groups)
    for (int sl = 0; sl < G.ns; ++sl) G.l64(0, sl).x = G.l64(0, sl).b = nullptr;
  if (res != MG_OK) return res;
  for (Group& G : h->groups) {
    res = upload_descriptors(h, G);
    if (res != MG_OK) return res;
  }
  if (!h->merges.empty()) {
    res = upload_merge_tables(h);
    if (res != MG_OK) return res;
  }
  HIPCHK(h, hipMemsetAsync(h->dstate, 0, (size_t)h->nprob * sizeof(SolveState), st));
  return sync_check(h);
}

// Common part of mg_setup and mg_setup_batched after the groups are formed.
mg_status setup_handle(mg_handle h, const mg_coeffs* coeffs, int32_t levels) {
  h->galerkin5 = h->kind == MG_COEF_CONST5 && h->opts.coarse_op == MG_COARSE_GALERKIN;
  if (h->galerkin5) h->oned = 1;
  h->line = line_dirs(h->opts.smoother);
  h->line_jac = line_jacobi(h->opts.smoother);
  h->ncol = (h->opts.smoother == MG_SMOOTH_JACOBI || h->line) ? 0 : (h->opts.smoother == MG_SMOOTH_RBGS ? 2 : 4);
  h->stream = static_cast<hipStream_t>(h->opts.stream);
  h->ncus = device_cus();
  HIPCHK(h, hipEventCreate(&h->ev0));
  HIPCHK(h, hipEventCreate(&h->ev1));
  HIPCHK(h, h->dalloc(&h->dstate, (size_t)h->nprob * sizeof(SolveState)));
  HIPCHK(h, h->dalloc(&h->dstate_res, sizeof(SolveState)));
  HIPCHK(h, h->dalloc(&h->dLres, sizeof(Level<double>)));
  h->hist_cap = 4097;
  h->dhist.assign(h->nprob, nullptr);
  for (int p = 0; p < h->nprob; ++p) HIPCHK(h, h->dalloc(&h->dhist[p], (size_t)h->hist_cap * sizeof(double)));

  // coefficient checks (read-only device pass)
  mg_coeffs folded{};
  if (h->kind == MG_COEF_CELL9) {
    HIPCHK(h, h->dalloc(&h->dcount, sizeof(int)));
    mg_status s = check_cell_coeffs(h, coeffs);
    if (s != MG_OK) return s;
    if (h->graded) {
      // the hierarchy takes the caller's cells folded with the cell widths
      const mg_grid& grid = h->groups[0].grid;
      const int ncx = grid.nx - 1;
      h->grows = h->oned ? 1 : (grid.periodic_y ? grid.ny : grid.ny - 1);
      HIPCHK(h, h->dalloc(&h->grx, h->hrx.size() * sizeof(double)));
      HIPCHK(h, h->dalloc(&h->gry, h->hry.size() * sizeof(double)));
      HIPCHK(h, hipMemcpyAsync(h->grx, h->hrx.data(), h->hrx.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
      HIPCHK(h, hipMemcpyAsync(h->gry, h->hry.data(), h->hry.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
      HIPCHK(h, h->dalloc(&h->gkx, (size_t)ncx * h->grows * sizeof(double)));
      HIPCHK(h, h->dalloc(&h->gky, (size_t)ncx * h->grows * sizeof(double)));
      HIPCHK(h, launch_graded_cells(coeffs->kx, coeffs->ky, h->in_oned, h->grx, h->gry, h->gkx, h->gky, ncx, h->grows,
                                    h->stream));
      folded = *coeffs;
      folded.kx = h->gkx;
      folded.ky = h->gky;
      folded.kx_1d_along_x = h->oned;
      coeffs = &folded;
      HIPCHK(h, hipStreamSynchronize(h->stream));  // the host ratio arrays stay, but settle the copies here
    }
  }
  HIPCHK(h, h->mixed() ? prepare_subcycle_lds<float>() : prepare_subcycle_lds<double>());
  if (h->line) HIPCHK(h, h->mixed() ? prepare_line_cr<float>() : prepare_line_cr<double>());
  HIPCHK(h, h->mixed() ? prepare_fused<float>() : prepare_fused<double>());
  for (Group& G : h->groups) {
    mg_status s = setup_group(h, G, coeffs, levels);
    if (s != MG_OK) return s;
  }
  // partial sums of a norm reduction: one per workgroup of the norm kernel or
  // of the finest post-pass when it carries the stopping test
  // (the autotuner's candidates included: at most one workgroup per 16 x 4 nodes)
  h->dpartial.assign(h->nprob, nullptr);
  for (const Group& G : h->groups) {
    size_t nparts = MAX_NORM_BLOCKS;
    nparts = std::max(nparts, (size_t)G.gpost[0].ntx * G.gpost[0].nty);
    nparts = std::max(nparts, (size_t)((G.shp[0].nx + 15) / 16) * ((G.shp[0].ny + 3) / 4));
    for (int s = 0; s < G.ns; ++s) HIPCHK(h, h->dalloc(&h->dpartial[G.probs[s]], nparts * sizeof(double)));
  }
  for (Group& G : h->groups) {
    mg_status s = upload_descriptors(h, G);
    if (s != MG_OK) return s;
  }
  mg_status s = sync_check(h);
  if (s != MG_OK) return s;
  s = build_merges(h);
  if (s != MG_OK) return s;
  s = tune_handle(h);
  if (s != MG_OK) return s;
  return build_graphs(h);
}

mg_status grow_history(mg_handle h, int need) {
  if (need <= h->hist_cap) return MG_OK;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int p = 0; p < h->nprob; ++p) {
    double* q = nullptr;
    HIPCHK(h, h->dalloc(&q, (size_t)need * sizeof(double)));
    h->dhist[p] = q;  // the old buffer stays owned by the handle until mg_destroy
  }
  h->hist_cap = need;
  return MG_OK;
}

// Points every problem's finest level at the caller's arrays, zeroes their
// Dirichlet boundaries, resets the stopping states and measures r0 (events
// start before the r0 measurement).
mg_status begin_solve(mg_handle h, const double* const* rhs, double* const* x, double tol) {
  hipStream_t st = h->stream;
  std::vector<SolveState> init(h->nprob);
  for (int p = 0; p < h->nprob; ++p) {
    init[p] = SolveState{};
    init[p].tol = tol;
    init[p].history = h->dhist[p];
    init[p].hist_cap = h->hist_cap;
    init[p].partial = h->dpartial[p];
  }
  HIPCHK(h, hipMemcpyAsync(h->dstate, init.data(), (size_t)h->nprob * sizeof(SolveState), hipMemcpyHostToDevice, st));
  for (Group& G : h->groups) {
    for (int s = 0; s < G.ns; ++s) {
      const int p = G.probs[s];
      G.l64(0, s).x = x[p];
      G.l64(0, s).b = const_cast<double*>(rhs[p]);
      const LevelShape& s0 = G.shp[0];
      HIPCHK(h, launch_zero_boundary(x[p], s0.nx, s0.ny, s0.nx, s0.py, st));
    }
    mg_status s = upload_descriptors(h, G);  // also waits for the state upload above
    if (s != MG_OK) return s;
  }
  if (!h->merges.empty()) {
    mg_status s = upload_merge_tables(h);
    if (s != MG_OK) return s;
  }
  HIPCHK(h, hipEventRecord(h->ev0, st));
  for (Group& G : h->groups)
    HIPCHK(h, launch_resnorm<double>(G.dL64, G.shp[0], NORM_INIT, nullptr, h->mixed() ? G.dL32 : nullptr,
                                     stencil_kind(h), h->oned, G.ns, st));
  return MG_OK;
}

// Replays the cycle graph until every problem stopped or max_cycles cycles
// were queued; reads the stopping states once per batch into `cur`.
mg_status run_cycles(mg_handle h, int max_cycles, double tol, std::vector<SolveState>& cur) {
  hipStream_t st = h->stream;
  cur.assign(h->nprob, SolveState{});
  int queued = 0, batch = 1;
  while (true) {
    const int nb = std::min(batch, max_cycles - queued);
    for (int k = 0; k + 8 <= nb; k += 8) HIPCHK(h, hipGraphLaunch(h->g8, st));
    for (int k = 0; k < nb % 8; ++k) HIPCHK(h, hipGraphLaunch(h->g1, st));
    queued += nb;
    for (int u : h->standalone)
      if (resid_fused(h, h->groups[u])) HIPCHK(h, tail_check(h, h->groups[u], st));
    HIPCHK(h, hipMemcpyAsync(cur.data(), h->dstate, (size_t)h->nprob * sizeof(SolveState), hipMemcpyDeviceToHost,
                             st));
    HIPCHK(h, hipStreamSynchronize(st));
    if (queued >= max_cycles) break;
    // predict the cycles still needed from the slowest running problem's latest factor
    int need = 0;
    bool running = false;
    for (const SolveState& s : cur) {
      if (s.done) continue;
      running = true;
      const double rho = s.prev > 0 ? s.last / s.prev : 0.0;
      const double goal = tol * s.r0;
      int n = std::min(2 * batch, 64);
      if (rho > 0.0 && rho < 1.0 && s.last > goal)
        n = (int)std::min(4096.0, std::max(1.0, std::ceil(std::log(goal / s.last) / std::log(rho))));
      need = std::max(need, n);
    }
    if (!running) break;
    batch = std::max(1, need);
  }
  return MG_OK;
}

mg_status status_of(const SolveState& s) {
  return s.done == 1 ? MG_OK : (s.done == 2 ? MG_DIVERGED : MG_NOT_CONVERGED);
}

void fill_info(const SolveState& s, float ms, mg_info* info) {
  info->status = status_of(s);
  info->cycles = s.cycles;
  info->res0 = s.r0;
  info->res = s.last;
  info->rel_res = s.r0 > 0 ? s.last / s.r0 : 0.0;
  info->rho_last = s.prev > 0 ? s.last / s.prev : 0.0;
  info->rho_mean = (s.cycles > 0 && s.r0 > 0 && s.last > 0) ? std::pow(s.last / s.r0, 1.0 / s.cycles) : 0.0;
  info->seconds = ms * 1e-3;
}

mg_status single_only(mg_handle h) {
  if (!h) return fail(nullptr, MG_EINVAL, "handle is NULL");
  if (h->batched) return fail(h, MG_EUNSUPPORTED, "handle was made by mg_setup_batched");
  return MG_OK;
}

mg_status finish_solve(mg_handle h, float* ms) {
  HIPCHK(h, hipEventRecord(h->ev1, h->stream));
  HIPCHK(h, hipEventSynchronize(h->ev1));
  HIPCHK(h, hipEventElapsedTime(ms, h->ev0, h->ev1));
  return MG_OK;
}

// Nested iteration on the hierarchy of type T (the one the cycles run on),
// its finest x zero and its finest b the right-hand side: restrictions down,
// the coarsest solve, then per level upwards the prolongation and one cycle,
// finally the prolongation into the finest x.  Every op is its own launch.
template <typename T>
hipError_t nested_pass(mg_handle h, Group& G, Level<T>* dL, Level<T>* dP, T omega, hipStream_t st) {
  const int c = G.nlev - 1;
  Gen g{h, G, 0};
  hipError_t e = hipSuccess;
  auto run = [&](int type, int l) { return run_op<T>(h, G, HostOp{type, l, 0, -1}, dL, dP, omega, st); };
  for (int l = 0; l < c; ++l)  // b_{l+1} = R b_l (x_l = 0), x_{l+1} = 0
    if ((e = run(H_DR, l)) != hipSuccess) return e;
  if ((e = run(H_COARSE, c)) != hipSuccess) return e;
  for (int l = c - 1; l >= 1; --l) {
    if ((e = run(H_PROLONG, l)) != hipSuccess) return e;  // x_l = P x_{l+1}
    std::vector<Abs> ops;
    g.expand(ops, l, h->opts.cycle);
    for (const Abs& a : ops)
      if ((e = run_op<T>(h, G, HostOp{a.type, a.level, a.arg, -1}, dL, dP, omega, st)) != hipSuccess) return e;
  }
  return c >= 1 ? run(H_PROLONG, 0) : hipSuccess;
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

int32_t mg_num_levels(mg_handle h) { return h && !h->groups.empty() ? h->groups[0].nlev : 0; }

mg_status mg_level_shape(mg_handle h, int32_t l, int32_t* nx, int32_t* ny) {
  if (!h || !nx || !ny) return fail(h, MG_EINVAL, "NULL argument");
  const Group& G = h->groups[0];
  if (l < 0 || l >= G.nlev) return fail(h, MG_EINVAL, "level out of range");
  *nx = G.shp[l].nx;
  *ny = G.shp[l].ny;
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
    if (grid->xs || grid->ys) return fail(nullptr, MG_EUNSUPPORTED, "refined grids (xs, ys) need MG_COEF_CELL9");
  } else if (coeffs->kind == MG_COEF_CELL9) {
    if (!coeffs->kx || !coeffs->ky) return fail(nullptr, MG_EINVAL, "kx and ky must be device arrays");
  } else {
    return fail(nullptr, MG_EINVAL, "unknown coefficient kind");
  }
  s = check_opts(opts, coeffs->kind);
  if (s != MG_OK) return s;
  if (levels < 0) return fail(nullptr, MG_EINVAL, "levels must be >= 0");
  if ((line_dirs(opts->smoother) & 2) && grid->periodic_y)
    return fail(nullptr, MG_EUNSUPPORTED, "line smoothers along a periodic direction (y lines with periodic_y)");

  mg_handle h = new mg_handle_s();
  h->opts = *opts;
  h->kind = coeffs->kind;
  h->in_oned = coeffs->kx_1d_along_x ? 1 : 0;
  h->oned = h->in_oned;
  if (grid->xs || grid->ys) {
    // cell widths over the equidistant width; the folded coefficients vary
    // along x only if the caller's do and y is not refined
    h->graded = true;
    const int ncx = grid->nx - 1, ncy = grid->periodic_y ? grid->ny : grid->ny - 1;
    const double hx0 = grid->lx / ncx, hy0 = grid->ly / ncy;
    h->hrx.assign(ncx, 1.0);
    h->hry.assign(grid->ys ? ncy : 1, 1.0);
    if (grid->xs)
      for (int i = 0; i < ncx; ++i) h->hrx[i] = (grid->xs[i + 1] - grid->xs[i]) / hx0;
    if (grid->ys)
      for (int j = 0; j < ncy; ++j) h->hry[j] = (grid->ys[j + 1] - grid->ys[j]) / hy0;
    if (grid->ys) h->oned = 0;
    if (!h->oned && h->hry.size() == 1) h->hry.assign(ncy, 1.0);
  }
  h->nprob = 1;
  h->eps_x.assign(1, coeffs->eps_x);
  h->eps_y.assign(1, coeffs->eps_y);
  h->groups.resize(1);
  h->groups[0].grid = *grid;
  h->groups[0].grid.xs = h->groups[0].grid.ys = nullptr;  // caller memory: not kept
  h->groups[0].ns = 1;
  h->groups[0].probs = {0};
  s = setup_handle(h, coeffs, levels);
  if (s != MG_OK) {
    g_thread_err = h->err;
    release(h);
    delete h;
    return s;
  }
  *out = h;
  return MG_OK;
}

mg_status mg_setup_batched(const mg_grid* grids, const mg_coeffs* coeffs, int32_t nprob, int32_t levels,
                           const mg_options* opts, mg_handle* out) {
  g_thread_err.clear();
  if (!out) return fail(nullptr, MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grids || !coeffs) return fail(nullptr, MG_EINVAL, "grids and coeffs must be host arrays");
  if (nprob < 1 || nprob > MAX_BATCH)
    return fail(nullptr, MG_EINVAL, "nprob must be in [1, " + std::to_string(MAX_BATCH) + "]");
  for (int p = 0; p < nprob; ++p) {
    mg_status s = check_grid(grids + p);
    if (s != MG_OK) return fail(nullptr, s, "problem " + std::to_string(p) + ": " + g_thread_err);
    if (coeffs[p].kind != MG_COEF_CONST5)
      return fail(nullptr, MG_EUNSUPPORTED, "batched solves take MG_COEF_CONST5 problems only");
    if (grids[p].xs || grids[p].ys) return fail(nullptr, MG_EUNSUPPORTED, "batched solves take equidistant grids");
    if (!(finite_pos(coeffs[p].eps_x) && finite_pos(coeffs[p].eps_y)))
      return fail(nullptr, MG_EINVAL, "problem " + std::to_string(p) + ": eps_x and eps_y must be finite and > 0");
  }
  mg_status s = check_opts(opts, MG_COEF_CONST5);
  if (s != MG_OK) return s;
  if (line_dirs(opts->smoother)) return fail(nullptr, MG_EUNSUPPORTED, "batched solves take point smoothers only");
  if (opts->coarse_op == MG_COARSE_GALERKIN)
    return fail(nullptr, MG_EUNSUPPORTED, "batched solves rediscretise their coarse operators");
  if (levels < 0) return fail(nullptr, MG_EINVAL, "levels must be >= 0");
  for (int p = 0; p < nprob; ++p)
    if (levels > max_levels(grids[p].nx, grids[p].ny, grids[p].periodic_y ? 1 : 0))
      return fail(nullptr, MG_EINVAL, "problem " + std::to_string(p) + ": grid cannot provide " +
                                          std::to_string(levels) + " levels");

  mg_handle h = new mg_handle_s();
  h->batched = true;
  h->opts = *opts;
  h->kind = MG_COEF_CONST5;
  h->nprob = nprob;
  h->eps_x.resize(nprob);
  h->eps_y.resize(nprob);
  // one group per distinct grid, largest grids first
  std::map<std::tuple<int, int, int, double, double>, int> key;
  std::vector<int> order(nprob);
  for (int p = 0; p < nprob; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (long)grids[a].nx * grids[a].ny > (long)grids[b].nx * grids[b].ny;
  });
  for (int p : order) {
    h->eps_x[p] = coeffs[p].eps_x;
    h->eps_y[p] = coeffs[p].eps_y;
    const auto k = std::make_tuple(grids[p].nx, grids[p].ny, grids[p].periodic_y, grids[p].lx, grids[p].ly);
    auto it = key.find(k);
    int g;
    if (it == key.end()) {
      g = (int)h->groups.size();
      key[k] = g;
      h->groups.emplace_back();
      h->groups[g].grid = grids[p];
      h->groups[g].ns = 0;
    } else {
      g = it->second;
    }
    h->groups[g].ns++;
    h->groups[g].probs.push_back(p);
  }
  s = setup_handle(h, nullptr, levels);
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
  mg_status s = single_only(h);
  if (s != MG_OK) return s;
  if (!rhs || !x) return fail(h, MG_EINVAL, "rhs and x must be device arrays");
  if (!(std::isfinite(tol) && tol > 0.0)) return fail(h, MG_EINVAL, "tol must be finite and > 0");
  if (max_cycles < 1) return fail(h, MG_EINVAL, "max_cycles must be >= 1");
  s = grow_history(h, max_cycles + 1);
  if (s != MG_OK) return s;
  const double* rr[1] = {rhs};
  double* xx[1] = {x};
  s = begin_solve(h, rr, xx, tol);
  if (s != MG_OK) return s;
  std::vector<SolveState> cur;
  s = run_cycles(h, max_cycles, tol, cur);
  if (s != MG_OK) return s;
  float ms = 0.f;
  s = finish_solve(h, &ms);
  if (s != MG_OK) return s;
  if (info) {
    fill_info(cur[0], ms, info);
    if (info->history)
      HIPCHK(h, hipMemcpy(info->history, h->dhist[0], (size_t)(cur[0].cycles + 1) * sizeof(double),
                          hipMemcpyDeviceToHost));
  }
  return status_of(cur[0]);
}

mg_status mg_solve_batched(mg_handle h, const double* const* rhs, double* const* x, double tol, int32_t max_cycles,
                           mg_info* info) {
  if (!h) return fail(nullptr, MG_EINVAL, "handle is NULL");
  if (!h->batched) return fail(h, MG_EUNSUPPORTED, "handle was made by mg_setup");
  if (!rhs || !x) return fail(h, MG_EINVAL, "rhs and x must be host arrays of device pointers");
  for (int p = 0; p < h->nprob; ++p)
    if (!rhs[p] || !x[p]) return fail(h, MG_EINVAL, "problem " + std::to_string(p) + ": NULL array");
  if (!(std::isfinite(tol) && tol > 0.0)) return fail(h, MG_EINVAL, "tol must be finite and > 0");
  if (max_cycles < 1) return fail(h, MG_EINVAL, "max_cycles must be >= 1");
  mg_status s = grow_history(h, max_cycles + 1);
  if (s != MG_OK) return s;
  s = begin_solve(h, rhs, x, tol);
  if (s != MG_OK) return s;
  std::vector<SolveState> cur;
  s = run_cycles(h, max_cycles, tol, cur);
  if (s != MG_OK) return s;
  float ms = 0.f;
  s = finish_solve(h, &ms);
  if (s != MG_OK) return s;
  mg_status worst = MG_OK;
  for (int p = 0; p < h->nprob; ++p) {
    if (info) {
      fill_info(cur[p], ms, info + p);
      if (info[p].history)
        HIPCHK(h, hipMemcpy(info[p].history, h->dhist[p], (size_t)(cur[p].cycles + 1) * sizeof(double),
                            hipMemcpyDeviceToHost));
    }
    worst = std::max(worst, status_of(cur[p]));
  }
  return worst;
}

mg_status mg_residual(mg_handle h, const double* rhs, const double* x, double* r, double* norm2) {
  mg_status s = single_only(h);
  if (s != MG_OK) return s;
  if (!rhs || !x || !norm2) return fail(h, MG_EINVAL, "rhs, x and norm2 must not be NULL");
  hipStream_t st = h->stream;
  const Group& G = h->groups[0];
  const LevelShape& s0 = G.shp[0];
  Level<double> L = G.L64[0];
  L.x = const_cast<double*>(x);
  L.b = const_cast<double*>(rhs);
  L.st = h->dstate_res;
  SolveState init{};
  init.partial = h->dpartial[0];
  HIPCHK(h, hipMemcpyAsync(h->dstate_res, &init, sizeof(SolveState), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(h->dLres, &L, sizeof(Level<double>), hipMemcpyHostToDevice, st));
  if (r) HIPCHK(h, hipMemsetAsync(r, 0, (size_t)s0.nx * s0.ny * sizeof(double), st));
  HIPCHK(h, launch_resnorm<double>(h->dLres, s0, NORM_RESID, r, nullptr, stencil_kind(h), h->oned, 1, st));
  SolveState cur{};
  HIPCHK(h, hipMemcpyAsync(&cur, h->dstate_res, sizeof(SolveState), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  *norm2 = cur.last;
  return MG_OK;
}

mg_status mg_pass_info(mg_handle h, int32_t level, int32_t which, int32_t* out) {
  mg_status s = single_only(h);
  if (s != MG_OK) return s;
  if (!out) return fail(h, MG_EINVAL, "out must not be NULL");
  if (which != 0 && which != 1) return fail(h, MG_EINVAL, "which must be 0 (pre-pass) or 1 (post-pass)");
  Group& G = h->groups[0];
  if (level < 0 || level >= G.nlev) return fail(h, MG_EINVAL, "level out of range");
  bool found = false;
  for (const HostOp& op : G.prog)
    if (op.type == (which == 0 ? H_PRE : H_POST) && op.level == level) found = true;
  if (!found) return fail(h, MG_EUNSUPPORTED, "no fused pass of that kind runs on this level");
  const TileGeom& g = which == 0 ? G.gpre[level] : G.gpost[level];
  out[0] = g.wide;
  out[1] = g.TX;
  out[2] = g.TY;
  out[3] = g.H;
  out[4] = g.ntx * g.nty;
  out[5] = h->ncol;
  out[6] = stencil_kind(h);
  out[7] = stencil_kind(h) == ST9 && h->oned ? 1 : 0;
  out[8] = level == 0 && which == 0 && resid_fused(h, G) ? 1 : 0;
  out[9] = g.Hy;
  return MG_OK;
}

mg_status mg_profile_pass(mg_handle h, const double* rhs, double* x, int32_t level, int32_t which, int32_t reps,
                          double* avg_us) {
  mg_status s = single_only(h);
  if (s != MG_OK) return s;
  if (!rhs || !x || !avg_us) return fail(h, MG_EINVAL, "rhs, x and avg_us must not be NULL");
  if (which < 0 || which > 2) return fail(h, MG_EINVAL, "which must be 0 (pre-pass), 1 (post-pass) or 2 (line sweep)");
  if (reps < 1 || reps > 100000) return fail(h, MG_EINVAL, "reps must be in [1, 100000]");
  Group& G = h->groups[0];
  if (level < 0 || level >= G.nlev) return fail(h, MG_EINVAL, "level out of range");
  const HostOp* found = nullptr;
  for (const HostOp& op : G.prog)
    if (op.type == (which == 0 ? H_PRE : (which == 1 ? H_POST : H_LINE)) && op.level == level && !found)
      found = &op;
  if (!found)
    return fail(h, MG_EUNSUPPORTED, which == 2 ? "no line sweep runs on this level" : "no fused pass of that kind runs on this level");
  hipStream_t st = h->stream;
  const double* rr[1] = {rhs};
  double* xx[1] = {x};
  s = begin_solve(h, rr, xx, 1e-300);  // descriptors, zero boundary, a running state
  if (s != MG_OK) return s;
  const int l = level;
  const int kind = stencil_kind(h);
  // the finest level of the mixed form runs its passes as an outer step of
  // `inner` cycles does: launch r as inner cycle r % inner
  const int inner = l == 0 && h->mixed() && G.mixed_fused ? inner_cycles(h) : 1;
  auto launch = [&](int r) -> hipError_t {
    const int c = r % inner;
    if (which == 2) {
      if (h->mixed()) return launch_line<float>(G.dL32 + l, G.shp[l], found->arg, (float)h->opts.omega, kind, 1, st);
      return launch_line<double>(G.dL64 + l, G.shp[l], found->arg, h->opts.omega, kind, 1, st);
    }
    if (h->mixed()) {
      // level 0 as the solve runs it: the first inner cycle's pre-pass from
      // a zero start (forming the residual when that is the solve's path),
      // the last one's post-pass adding e into the FP64 iterate (e left for
      // the next pre-pass), the others keeping e
      const bool zs = l == 0 && mixed_zero_start(h, G);
      if (which == 0)
        return launch_pre<float>(G.dL32 + l, G.dL32 + l + 1, G.gpre[l], h->opts.nu_pre, h->ncol,
                                 (float)relax(h), kind, h->oned, l == 0, 1, st,
                                 zs && c == 0 ? (resid_fused(h, G) ? PRE_RESID : PRE_ZERO) : PRE_LOAD, G.dL64);
      int mode = zs && found->arg == POST_MIXED ? POST_MIXED_KEEP : found->arg;
      if (c + 1 < inner) mode = POST_PLAIN;
      return launch_post<float>(G.dL32 + l, G.dL32 + l + 1, G.gpost[l], h->opts.nu_post, h->ncol,
                                (float)relax(h), mode, G.dL64, kind, h->oned, l == 0, 1, st, false);
    }
    if (which == 0)
      return launch_pre<double>(G.dL64 + l, G.dL64 + l + 1, G.gpre[l], h->opts.nu_pre, h->ncol, relax(h),
                                kind, h->oned, l == 0, 1, st);
    return launch_post<double>(G.dL64 + l, G.dL64 + l + 1, G.gpost[l], h->opts.nu_post, h->ncol, relax(h),
                               found->arg, G.dL64, kind, h->oned, l == 0, 1, st, false);
  };
  HIPCHK(h, launch(inner - 1));
  HIPCHK(h, hipEventRecord(h->ev0, st));
  for (int r = 0; r < reps; ++r) HIPCHK(h, launch(r));
  HIPCHK(h, hipEventRecord(h->ev1, st));
  HIPCHK(h, hipEventSynchronize(h->ev1));
  float ms = 0.f;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
  *avg_us = 1e3 * ms / reps;
  return MG_OK;
}

mg_status mg_update_coeffs(mg_handle h, const mg_coeffs* coeffs) {
  mg_status s = single_only(h);
  if (s != MG_OK) return s;
  if (!coeffs) return fail(h, MG_EINVAL, "coeffs is NULL");
  if (h->kind != MG_COEF_CELL9 || coeffs->kind != MG_COEF_CELL9)
    return fail(h, MG_EINVAL, "coefficient update needs cell coefficients, at setup and now");
  if ((coeffs->kx_1d_along_x ? 1 : 0) != h->in_oned) return fail(h, MG_EINVAL, "kx_1d_along_x differs from setup");
  if (!coeffs->kx || !coeffs->ky) return fail(h, MG_EINVAL, "kx and ky must be device arrays");
  Group& G = h->groups[0];
  const Level<double>& L0 = G.l64(0, 0);
  if (L0.kcx && L0.kcx == L0.kcy && coeffs->kx != coeffs->ky)
    return fail(h, MG_EINVAL, "kx and ky were one array at setup and must be one array here");
  s = check_cell_coeffs(h, coeffs);
  if (s != MG_OK) return s;
  mg_coeffs folded = *coeffs;
  if (h->graded) {  // fold the new cells with the cell widths, as at setup
    HIPCHK(h, launch_graded_cells(coeffs->kx, coeffs->ky, h->in_oned, h->grx, h->gry, h->gkx, h->gky,
                                  G.grid.nx - 1, h->grows, h->stream));
    folded.kx = h->gkx;
    folded.ky = h->gky;
    folded.kx_1d_along_x = h->oned;
    coeffs = &folded;
  }
  HIPCHK(h, assemble_cell9(h, G, coeffs));
  if (h->line) HIPCHK(h, assemble_line_factors(h, G));
  return assemble_coarsest(h, G);
}

mg_status mg_start_nested(mg_handle h, const double* rhs, double* x) {
  mg_status s = single_only(h);
  if (s != MG_OK) return s;
  if (!rhs || !x) return fail(h, MG_EINVAL, "rhs and x must be device arrays");
  Group& G = h->groups[0];
  const LevelShape& s0 = G.shp[0];
  hipStream_t st = h->stream;
  HIPCHK(h, hipMemsetAsync(x, 0, (size_t)s0.nx * s0.ny * sizeof(double), st));
  if (h->mixed()) {
    const Level<float>& E = G.l32(0, 0);
    HIPCHK(h, hipMemsetAsync(E.x, 0, (size_t)E.pitch * s0.ny * sizeof(float), st));
  }
  const double* rr[1] = {rhs};
  double* xx[1] = {x};
  s = begin_solve(h, rr, xx, 1e-300);  // descriptors; r0 = ||b|| (mixed: the FP32 finest rhs = (float) b)
  if (s != MG_OK) return s;
  if (h->mixed()) {
    HIPCHK(h, nested_pass<float>(h, G, G.dL32, G.dP32, (float)relax(h), st));
    HIPCHK(h, launch_outer_update(G.dL64, G.dL32, s0, 1, st));  // x = (double) e, e = 0
  } else {
    HIPCHK(h, nested_pass<double>(h, G, G.dL64, G.dP64, relax(h), st));
  }
  return sync_check(h);
}

mg_status mg_coeff_grad(mg_handle h, const double* u, const double* lam, double* dL_dk) {
  mg_status s = single_only(h);
  if (s != MG_OK) return s;
  if (h->kind != MG_COEF_CELL9) return fail(h, MG_EUNSUPPORTED, "coefficient gradient needs MG_COEF_CELL9");
  if (h->graded) return fail(h, MG_EUNSUPPORTED, "coefficient gradient on a refined grid is not built");
  if (!u || !lam || !dL_dk) return fail(h, MG_EINVAL, "u, lam and dL_dk must be device arrays");
  const Group& G = h->groups[0];
  const LevelShape& s0 = G.shp[0];
  HIPCHK(h, launch_coeff_grad(u, lam, dL_dk, s0.nx, s0.ny, s0.py, G.hx[0], G.hy[0], h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return MG_OK;
}

mg_status mg_batch_schedule(mg_handle h, int32_t* out) {
  if (!h || !out) return fail(h, MG_EINVAL, "NULL argument");
  int in_merges = 0;
  for (const Merge& M : h->merges) in_merges += (int)M.groups.size();
  out[0] = (int32_t)h->merges.size();
  out[1] = in_merges;
  out[2] = (int32_t)h->standalone.size();
  out[3] = h->graph_nodes;
  return MG_OK;
}

mg_status mg_destroy(mg_handle h) {
  if (!h) return MG_OK;
  release(h);
  delete h;
  return MG_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------- residual without allocation
//
// mg_residual_noalloc: the residual and its norm (the kernels of mg_residual)
// for callers that cannot allocate device memory.  Its device scratch -- the
// finest-level descriptor, the norm state and the per-workgroup partial sums
// of the norm reduction -- lives in one file-scope device array per GPU,
// reached through the address hipGetSymbolAddress gives on that device.

namespace {

constexpr size_t NOALLOC_DESC_OFF = 0;
constexpr size_t NOALLOC_STATE_OFF = 512;
constexpr size_t NOALLOC_PARTIAL_OFF = 1024;
constexpr size_t NOALLOC_SCRATCH_BYTES = NOALLOC_PARTIAL_OFF + sizeof(double) * MAX_NORM_BLOCKS;  // 9 KiB
static_assert(sizeof(Level<double>) <= NOALLOC_STATE_OFF - NOALLOC_DESC_OFF, "descriptor slot too small");
static_assert(sizeof(SolveState) <= NOALLOC_PARTIAL_OFF - NOALLOC_STATE_OFF, "state slot too small");

// Largest stored grid side the call accepts: the norm reduction's partial
// sums (at most MAX_NORM_BLOCKS, however many rows) then fit the scratch.
constexpr int NOALLOC_MAX_SIDE = 65537;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Writes the descriptor and a cleared norm state into the scratch (kernel
// arguments, so nothing is copied from host memory).
__global__ void k_noalloc_init(Level<double>* dL, SolveState* dS, Level<double> L, double* partial) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  SolveState s{};
  s.partial = partial;
  *dS = s;
  *dL = L;
}

}  // namespace

extern "C" {

mg_status mg_residual_noalloc(const mg_grid* grid, const mg_coeffs* coeffs, const double* rhs, const double* x,
                              double* r, double* norm2, void* stream) {
  g_thread_err.clear();
  mg_status s = check_grid(grid);
  if (s != MG_OK) return s;
  if (grid->nx > NOALLOC_MAX_SIDE || grid->ny > NOALLOC_MAX_SIDE)
    return fail(nullptr, MG_EINVAL,
                "mg_residual_noalloc: nx and ny must be at most " + std::to_string(NOALLOC_MAX_SIDE) +
                    " (the norm's partial sums must fit its fixed scratch of " +
                    std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes)");
  if (!coeffs) return fail(nullptr, MG_EINVAL, "coeffs is NULL");
  if (!rhs || !x || !norm2) return fail(nullptr, MG_EINVAL, "rhs, x and norm2 must not be NULL");
  if (grid->xs || grid->ys) return fail(nullptr, MG_EUNSUPPORTED, "mg_residual_noalloc: refined grids need a handle");
  const int py = grid->periodic_y ? 1 : 0;
  const double hx = grid->lx / (grid->nx - 1);
  const double hy = py ? grid->ly / grid->ny : grid->ly / (grid->ny - 1);
  Level<double> L{};
  L.x = const_cast<double*>(x);
  L.b = const_cast<double*>(rhs);
  L.nx = grid->nx;
  L.ny = grid->ny;
  L.pitch = grid->nx;
  L.py = py;
  bool oned = false;
  if (coeffs->kind == MG_COEF_CONST5) {
    if (!(finite_pos(coeffs->eps_x) && finite_pos(coeffs->eps_y)))
      return fail(nullptr, MG_EINVAL, "eps_x and eps_y must be finite and > 0");
    L.kind = ST5;
    L.cx = coeffs->eps_x / (hx * hx);
    L.cy = coeffs->eps_y / (hy * hy);
    L.dg = 2.0 * (L.cx + L.cy);
    L.inv_dg = 1.0 / L.dg;
  } else if (coeffs->kind == MG_COEF_CELL9) {
    if (!coeffs->kx || !coeffs->ky) return fail(nullptr, MG_EINVAL, "kx and ky must be device arrays");
    // the couplings are formed from the caller's cells at every node
    oned = coeffs->kx_1d_along_x != 0;
    L.kind = ST9;
    L.kcx = coeffs->kx;
    L.kcy = coeffs->ky;
    L.kcpitch = oned ? 0 : grid->nx - 1;
    const double ax = 1.0 / (hx * hx), ay = 1.0 / (hy * hy);
    L.kc3x = ax / 3.0;
    L.kc3y = ay / 3.0;
    L.kc6x = ax / 6.0;
    L.kc6y = ay / 6.0;
  } else {
    return fail(nullptr, MG_EINVAL, "unknown coefficient kind");
  }
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess)
    return fail(nullptr, MG_EDEVICE, std::string("mg_residual_noalloc: scratch address: ") + hipGetErrorString(e));
  unsigned char* sp = static_cast<unsigned char*>(base);
  Level<double>* dL = reinterpret_cast<Level<double>*>(sp + NOALLOC_DESC_OFF);
  SolveState* dS = reinterpret_cast<SolveState*>(sp + NOALLOC_STATE_OFF);
  double* partial = reinterpret_cast<double*>(sp + NOALLOC_PARTIAL_OFF);
  L.st = dS;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const LevelShape s0{grid->nx, grid->ny, py, py ? grid->ny : grid->ny - 2};
#define NOALLOC_CHK(call)                                                                              \
  do {                                                                                                 \
    hipError_t e_ = (call);                                                                            \
    if (e_ != hipSuccess)                                                                              \
      return fail(nullptr, MG_EDEVICE, std::string("mg_residual_noalloc: ") + #call + ": " + hipGetErrorString(e_)); \
  } while (0)
  hipLaunchKernelGGL(k_noalloc_init, dim3(1), dim3(64), 0, st, dL, dS, L, partial);
  NOALLOC_CHK(hipGetLastError());
  // r: Dirichlet boundary nodes 0 (a fill kernel), every unknown written below
  if (r) NOALLOC_CHK(launch_zero_boundary(r, grid->nx, grid->ny, grid->nx, py, st));
  NOALLOC_CHK(launch_resnorm<double>(dL, s0, NORM_RESID, r, nullptr, L.kind, oned, 1, st));
  SolveState cur{};
  NOALLOC_CHK(hipMemcpyAsync(&cur, dS, sizeof(SolveState), hipMemcpyDeviceToHost, st));
  NOALLOC_CHK(hipStreamSynchronize(st));
#undef NOALLOC_CHK
  *norm2 = cur.last;
  return MG_OK;
}

}  // extern "C"
