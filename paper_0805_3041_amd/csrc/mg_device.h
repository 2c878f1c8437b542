// Device-side data structures and per-node arithmetic of the multigrid cycle.
//
// Every kernel (multi-workgroup sweeps on fine levels, the single-workgroup
// coarse-level interpreter, the fused tile kernels) computes a node's new
// value through the inline functions below, so a node gets the same
// floating-point expression whichever kernel updates it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mg {

// Pointer into LDS.  Written with the explicit address space so that every
// access compiles to ds_read/ds_write rather than flat instructions.
#define MG_LDS __attribute__((address_space(3)))

template <typename T>
__device__ __forceinline__ MG_LDS T* lds_cast(void* p) {
  return (MG_LDS T*)(p);
}

// Per-problem solve state, in device memory.  Written only by the last
// workgroup of a residual-norm kernel; read by every cycle kernel, which
// returns at once when `done` is set.
struct SolveState {
  double r0;              // ||b - A x0||
  double tol;             // relative tolerance
  double last;            // latest residual norm
  double prev;            // residual norm one cycle before `last`
  double* history;        // residual norms, index = cycle count
  int hist_cap;           // entries available in history
  int done;               // 0 running, 1 converged, 2 diverged
  int cycles;             // completed cycles
  unsigned int counter;   // workgroups finished in the running norm reduction
  double* partial;        // per-workgroup partial sums of the running norm
  int pending;            // the iterate changed since its last stopping test
};

enum StencilKind { ST5 = 0, ST9 = 1 };

// One level of one problem.  Stored nodes [ny][pitch]; Dirichlet x (and y
// unless py) boundary nodes hold 0 and are never written.
template <typename T>
struct Level {
  T* x;                   // iterate (or coarse correction)
  T* b;                   // right-hand side (restricted defect on coarse levels)
  T* t;                   // scratch of the same shape (Jacobi ping-pong)
  int nx, ny, pitch, py;  // stored shape, row pitch in elements, periodic y
  int kind;               // ST5 or ST9
  T cx, cy, dg;           // ST5: A x = dg x_p - cx (x_w + x_e) - cy (x_s + x_n)
  T inv_dg;               // ST5: 1 / dg
  const T* band;          // ST9: bands C, E, N, NE, NW, D = 1/C, each `bstride` apart
  int bpitch;             // ST9: band row pitch (0: one row for every j)
  int bstride;
  SolveState* st;         // owning problem's state
  T* lcp[2];              // line smoothers: per direction (0 x-lines, 1 y-lines) the Thomas factors
  T* lid[2];              //   c_n / den_n and 1 / den_n of every node's line, [ny][pitch]
  T* lr;                  //   forward-sweep values of the running line solve, [ny][pitch]
  // Finest level of a problem whose Q1 coefficients vary over the cells in
  // both directions, when the coarse-level interpreter does not run it: the
  // per-cell kx and ky ([ncy][kcpitch], cell (i, j) spanning nodes i..i+1,
  // j..j+1; one array when kx and ky are the same).  Kernels form a node's
  // couplings from its four cells (cell_coefs) instead of reading the six
  // bands.  Null elsewhere.
  const T* kcx;
  const T* kcy;
  int kcpitch;
  T kc3x, kc3y, kc6x, kc6y;  // 1/(3 hx^2), 1/(3 hy^2), 1/(6 hx^2), 1/(6 hy^2)
  // Adaptive coarse-correction weight omega_l of this level (device scalar
  // written by the energy reduction before each correction); null: the
  // correction is added with weight 1.
  T* wl;
};

// Host-built op of the coarse-level interpreter (one workgroup runs a list).
enum OpType {
  OP_COLOR = 0,     // Gauss-Seidel update of colour `arg` on `level`
  OP_JACOBI = 1,    // damped Jacobi x -> t (arg = 0) or t -> x (arg = 1)
  OP_COPY = 2,      // x <- t on `level`
  OP_DR = 3,        // restrict the defect of `level` into b of level+1, zero x of level+1
  OP_PROLONG = 4,   // x(level) += P x(level+1) (arg 1: times the level's adaptive omega_l)
  OP_COARSE = 5,    // exact solve on the coarsest `level`
  OP_LINE = 6,      // line sweep on `level`, arg as line_arg
  OP_OMEGA = 7,     // adaptive omega_l of `level` from its x, b and the correction on level+1
  OP_SMOOTH = 8,    // Gauss-Seidel sweeps (every colour in order) on `level`, with transfers (SmoothFlags)
};

// OP_SMOOTH arg: the number of sweeps (bits 0-4); SM_PRO: the level's
// coarse-grid correction is added first (SM_WTD: times the level's omega_l);
// SM_DR: the defect is restricted into level + 1 after the sweeps.
enum SmoothFlags {
  SM_NSW = 31,
  SM_PRO = 32,
  SM_WTD = 64,
  SM_DR = 128,
};

// Argument of a line-smoothing op: bit 0 direction (0: lines along x, 1:
// along y), bit 1 Jacobi (TRI) instead of Gauss-Seidel (GSTRI), bits 2+ the
// line colour (Gauss-Seidel: lines whose stored index has that parity) or the
// Jacobi ping-pong direction (0: x -> t, 1: t -> x).
constexpr int line_arg(int dir, bool jacobi, int sel) { return dir | ((jacobi ? 1 : 0) << 1) | (sel << 2); }

struct DOp {
  int type, level, arg, pad;
};

__device__ __forceinline__ int wrap_dn(int j, int n, int py) { return (py && j == 0) ? n - 1 : j - 1; }
__device__ __forceinline__ int wrap_up(int j, int n, int py) { return (py && j == n - 1) ? 0 : j + 1; }

// First and last stored row that carries unknowns.
template <typename T>
__device__ __forceinline__ int row_lo(const Level<T>& L) { return L.py ? 0 : 1; }
template <typename T>
__device__ __forceinline__ int row_hi(const Level<T>& L) { return L.py ? L.ny - 1 : L.ny - 2; }

template <typename T>
__device__ __forceinline__ const T* bandp(const Level<T>& L, int k) { return L.band + (size_t)k * L.bstride; }

// ---------------------------------------------------------------- x access
// The arithmetic below reads x through an accessor: at(di, dj) is the value
// at node (i + di, j + dj) of the node being updated (rows already wrapped).

// Global array, rows jm, j, jp given by pointers already offset to column i.
template <typename T>
struct GX {
  const T* rm;
  const T* r0;
  const T* rp;
  __device__ __forceinline__ T at(int di, int dj) const { return dj < 0 ? rm[di] : (dj > 0 ? rp[di] : r0[di]); }
};

// Same, but a Dirichlet boundary node reads as 0 whatever is stored there
// (used where x comes from the caller).
template <typename T>
struct GXMasked {
  GX<T> g;
  int i, j, nx, ny, py;
  __device__ __forceinline__ T at(int di, int dj) const {
    const int ii = i + di;
    const int jj = j + dj;
    if (ii == 0 || ii == nx - 1 || (!py && (jj == 0 || jj == ny - 1))) return (T)0;
    return g.at(di, dj);
  }
};

// Division by a small positive divisor fixed for a whole loop (a < 2^22):
// float reciprocal, then a one-step correction.
struct FDiv {
  int d;
  float inv;
  __device__ __forceinline__ explicit FDiv(int dd) : d(dd), inv(1.0f / (float)dd) {}
  __device__ __forceinline__ int q(int a) const {
    int r = (int)((float)a * inv);
    if (r * d > a) --r;
    else if ((r + 1) * d <= a) ++r;
    return r;
  }
};

// LDS rows jm, j, jp, already offset to column i.
template <typename T>
struct LX3 {
  const MG_LDS T* rm;
  const MG_LDS T* r0;
  const MG_LDS T* rp;
  __device__ __forceinline__ T at(int di, int dj) const { return dj < 0 ? rm[di] : (dj > 0 ? rp[di] : r0[di]); }
};

// LDS tile with row pitch W; p points at the node itself.
template <typename T>
struct LXW {
  const MG_LDS T* p;
  int W;
  __device__ __forceinline__ T at(int di, int dj) const { return p[dj * W + di]; }
};

template <typename T>
__device__ __forceinline__ GX<T> gx(const T* x, int pitch, int i, int j, int jm, int jp) {
  return GX<T>{x + (size_t)jm * pitch + i, x + (size_t)j * pitch + i, x + (size_t)jp * pitch + i};
}

// ---------------------------------------------------------------- arithmetic
// Every kernel computes a node's value with these functions.  A node's x
// neighbourhood and (9-point) coefficients are first gathered into registers
// (so a thread can issue the loads of several nodes before using any), then
// combined by the value functions below, always in the same order.

// x around node p: c = p, then the 4 edge and 4 corner neighbours.
template <typename T>
struct Nbr {
  T c, w, e, s, n, sw, se, nw, ne;
};

// a_pq of node p for its 9 couplings (symmetric band storage resolved) and
// D = 1 / a_pp.
template <typename T>
struct Cf {
  T C, Ep, Ew, Np, Ns, NEp, NEsw, NWp, NWse, D;
};

// Band index of the inverse diagonal.
constexpr int BAND_D = 5;
constexpr int NBANDS = 6;

// Stencil kind known at compile time (ST5, ST9) or read from the level (KDYN).
constexpr int KDYN = -1;
template <int K, typename T>
__device__ __forceinline__ bool is5(const Level<T>& L) {
  return K == ST5 ? true : (K == ST9 ? false : L.kind == ST5);
}

// Nodes a thread updates back to back in one sweep: all their loads are
// issued before the first value is computed (nodes of one sweep never read
// each other).  Fewer for 9-point operators, which need more registers.
__host__ __device__ constexpr int nbatch(int K) { return K == ST5 ? 4 : 2; }

template <int K = KDYN, typename T, typename X>
__device__ __forceinline__ Nbr<T> gather(const Level<T>& L, const X& x, bool centre) {
  Nbr<T> v{};
  if (centre) v.c = x.at(0, 0);
  v.w = x.at(-1, 0);
  v.e = x.at(1, 0);
  v.s = x.at(0, -1);
  v.n = x.at(0, 1);
  if (!is5<K>(L)) {
    v.sw = x.at(-1, -1);
    v.se = x.at(1, -1);
    v.nw = x.at(-1, 1);
    v.ne = x.at(1, 1);
  }
  return v;
}

// Coefficients at interior node (i, j) of a level with per-cell kx, ky:
// the bilinear element's couplings summed over the node's four cells SW
// (i-1, jm), SE (i, jm), NW (i-1, j), NE (i, j).  Each coupling collects the
// cells its two nodes share (east: SE and NE, north: NW and NE, the
// diagonals one cell each), the diagonal all four, with the per-cell terms
// of the element matrix kx/hx^2 K1 (x) M1 + ky/hy^2 M1 (x) K1 (K1 = [1 -1;
// -1 1], M1 = [1/3 1/6; 1/6 1/3]): diagonal (cx + cy)/3, east -cx/3 + cy/6,
// north cx/6 - cy/3, corner -(cx + cy)/6, cx = kx/hx^2, cy = ky/hy^2.  The
// same operator as the bands k_q1_bands assembles, up to rounding.
template <typename T>
__device__ __forceinline__ Cf<T> cell_coefs(const Level<T>& L, int i, int j, int jm) {
  const T* xs = L.kcx + (size_t)jm * L.kcpitch + i - 1;
  const T* xn = L.kcx + (size_t)j * L.kcpitch + i - 1;
  const T* ys = L.kcy + (size_t)jm * L.kcpitch + i - 1;
  const T* yn = L.kcy + (size_t)j * L.kcpitch + i - 1;
  const T xsw = xs[0], xse = xs[1], xnw = xn[0], xne = xn[1];
  const T ysw = ys[0], yse = ys[1], ynw = yn[0], yne = yn[1];
  Cf<T> c;
  c.C = L.kc3x * ((xsw + xse) + (xnw + xne)) + L.kc3y * ((ysw + yse) + (ynw + yne));
  c.Ep = L.kc6y * (yse + yne) - L.kc3x * (xse + xne);
  c.Ew = L.kc6y * (ysw + ynw) - L.kc3x * (xsw + xnw);
  c.Np = L.kc6x * (xnw + xne) - L.kc3y * (ynw + yne);
  c.Ns = L.kc6x * (xsw + xse) - L.kc3y * (ysw + yse);
  c.NEp = -(L.kc6x * xne + L.kc6y * yne);
  c.NEsw = -(L.kc6x * xsw + L.kc6y * ysw);
  c.NWp = -(L.kc6x * xnw + L.kc6y * ynw);
  c.NWse = -(L.kc6x * xse + L.kc6y * yse);
  c.D = (T)1 / c.C;
  return c;
}

// Coefficients at interior node (i, j); jm is j's wrapped lower row.  From
// the four cells where the level keeps them (every kernel that can run the
// finest level then forms the same values), else from the bands.  CELLS
// false leaves the cell path out of kernels that only run coarser levels
// (the coarse-level interpreter, whose registers it would spill).
template <int K = KDYN, bool CELLS = true, typename T>
__device__ __forceinline__ Cf<T> coefs(const Level<T>& L, int i, int j, int jm) {
  Cf<T> c{};
  if (is5<K>(L)) return c;
  if constexpr (CELLS) {
    if (L.kcx) return cell_coefs(L, i, j, jm);
  }
  const size_t rp = (size_t)j * L.bpitch, rs = (size_t)jm * L.bpitch;
  c.C = bandp(L, 0)[rp + i];
  c.Ep = bandp(L, 1)[rp + i];
  c.Ew = bandp(L, 1)[rp + i - 1];
  c.Np = bandp(L, 2)[rp + i];
  c.Ns = bandp(L, 2)[rs + i];
  c.NEp = bandp(L, 3)[rp + i];
  c.NEsw = bandp(L, 3)[rs + i - 1];
  c.NWp = bandp(L, 4)[rp + i];
  c.NWse = bandp(L, 4)[rs + i + 1];
  c.D = bandp(L, BAND_D)[rp + i];
  return c;
}

// Sum over the neighbours q != p of a_pq x_q, as one chain of fused
// multiply-adds in a fixed order.
template <int K = KDYN, typename T>
__device__ __forceinline__ T offd(const Level<T>& L, const Cf<T>& a, const Nbr<T>& v) {
  if (is5<K>(L)) return -fma(L.cx, v.w + v.e, L.cy * (v.s + v.n));
  T s = a.Ep * v.e;
  s = fma(a.Ew, v.w, s);
  s = fma(a.Np, v.n, s);
  s = fma(a.Ns, v.s, s);
  s = fma(a.NEp, v.ne, s);
  s = fma(a.NEsw, v.sw, s);
  s = fma(a.NWp, v.nw, s);
  s = fma(a.NWse, v.se, s);
  return s;
}

template <int K = KDYN, typename T>
__device__ __forceinline__ T inv_diag(const Level<T>& L, const Cf<T>& a) {
  return is5<K>(L) ? L.inv_dg : a.D;
}

// Gauss-Seidel value: (b_p - sum_{q != p} a_pq x_q) / a_pp.
template <int K = KDYN, typename T>
__device__ __forceinline__ T gs_v(const Level<T>& L, const Cf<T>& a, const Nbr<T>& v, T bp) {
  return (bp - offd<K>(L, a, v)) * inv_diag<K>(L, a);
}

// Relaxed Gauss-Seidel value (SOR, C = D + omega L in colour order): the
// node's old value *xp moved by omega towards its Gauss-Seidel value gs;
// omega = 1 returns gs itself without loading the old value (omega is
// uniform, so plain Gauss-Seidel sweeps issue no extra load).
template <typename T, typename P>
__device__ __forceinline__ T sor_v(T gs, P xp, T omega) {
  if (omega == (T)1) return gs;
  const T xc = *xp;
  return fma(omega, gs - xc, xc);
}

// Defect b_p - (A x)_p.
template <int K = KDYN, typename T>
__device__ __forceinline__ T defect_v(const Level<T>& L, const Cf<T>& a, const Nbr<T>& v, T bp) {
  const T dg = is5<K>(L) ? L.dg : a.C;
  return bp - fma(dg, v.c, offd<K>(L, a, v));
}

// Damped Jacobi value: x_p + omega (b - A x)_p / a_pp.
template <int K = KDYN, typename T>
__device__ __forceinline__ T jac_v(const Level<T>& L, const Cf<T>& a, const Nbr<T>& v, T bp, T omega) {
  return fma(omega * defect_v<K>(L, a, v, bp), inv_diag<K>(L, a), v.c);
}

// Accessor forms (gather, then the value functions above).
template <int K = KDYN, bool CELLS = true, typename T, typename X>
__device__ __forceinline__ T gs_val(const Level<T>& L, const X& x, T bp, int i, int j, int jm) {
  return gs_v<K>(L, coefs<K, CELLS>(L, i, j, jm), gather<K>(L, x, false), bp);
}

template <int K = KDYN, bool CELLS = true, typename T, typename X>
__device__ __forceinline__ T defect_val(const Level<T>& L, const X& x, T bp, int i, int j, int jm) {
  return defect_v<K>(L, coefs<K, CELLS>(L, i, j, jm), gather<K>(L, x, true), bp);
}

template <int K = KDYN, bool CELLS = true, typename T, typename X>
__device__ __forceinline__ T jac_val(const Level<T>& L, const X& x, T bp, int i, int j, int jm, T omega) {
  return jac_v<K>(L, coefs<K, CELLS>(L, i, j, jm), gather<K>(L, x, true), bp, omega);
}

// Full weighting of a 3x3 block of fine defects d[row][col] (row 0 = south):
// (1/16) [1 2 1; 2 4 2; 1 2 1].
template <typename T>
__device__ __forceinline__ T fw_combine(T s0, T s1, T s2) {  // s_r = row r's (1/4, 1/2, 1/4) combination
  return (T)0.25 * (s0 + s2) + (T)0.5 * s1;
}
template <typename T>
__device__ __forceinline__ T fw_row(T dw, T dc, T de) {
  return (T)0.25 * (dw + de) + (T)0.5 * dc;
}

// Convenience wrappers over a global array.
template <bool CELLS = true, typename T>
__device__ __forceinline__ T gs_value(const Level<T>& L, const T* __restrict__ x, const T* __restrict__ b,
                                      int i, int j, int jm, int jp) {
  return gs_val<KDYN, CELLS>(L, gx(x, L.pitch, i, j, jm, jp), b[(size_t)j * L.pitch + i], i, j, jm);
}

template <bool CELLS = true, typename T>
__device__ __forceinline__ T defect_at(const Level<T>& L, const T* __restrict__ x, const T* __restrict__ b,
                                       int i, int j, int jm, int jp) {
  return defect_val<KDYN, CELLS>(L, gx(x, L.pitch, i, j, jm, jp), b[(size_t)j * L.pitch + i], i, j, jm);
}

template <typename T>
__device__ __forceinline__ T defect_masked(const Level<T>& L, const T* __restrict__ x, const T* __restrict__ b,
                                           int i, int j, int jm, int jp) {
  GXMasked<T> m{gx(x, L.pitch, i, j, jm, jp), i, j, L.nx, L.ny, L.py};
  return defect_val(L, m, b[(size_t)j * L.pitch + i], i, j, jm);
}

template <bool CELLS = true, typename T>
__device__ __forceinline__ T jacobi_value(const Level<T>& L, const T* __restrict__ x, const T* __restrict__ b,
                                          int i, int j, int jm, int jp, T omega) {
  return jac_val<KDYN, CELLS>(L, gx(x, L.pitch, i, j, jm, jp), b[(size_t)j * L.pitch + i], i, j, jm, omega);
}

// Full-weighting restriction of the fine defect at coarse node (I, J),
// centred on fine node (2I, 2J).
template <bool CELLS = true, typename T>
__device__ __forceinline__ T restrict_defect(const Level<T>& F, const T* __restrict__ x, const T* __restrict__ b,
                                             int I, int J) {
  const int i0 = 2 * I;
  const int j0 = 2 * J;
  const int jm = wrap_dn(j0, F.ny, F.py);
  const int jp = wrap_up(j0, F.ny, F.py);
  const int rows[3] = {jm, j0, jp};
  T acc[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int j = rows[r];
    const int jjm = wrap_dn(j, F.ny, F.py);
    const int jjp = wrap_up(j, F.ny, F.py);
    const T dw = defect_at<CELLS>(F, x, b, i0 - 1, j, jjm, jjp);
    const T dc = defect_at<CELLS>(F, x, b, i0, j, jjm, jjp);
    const T de = defect_at<CELLS>(F, x, b, i0 + 1, j, jjm, jjp);
    acc[r] = fw_row(dw, dc, de);
  }
  return fw_combine(acc[0], acc[1], acc[2]);
}

// Bilinear interpolation from the coarse values around fine node (i, j):
// a00 = e(I, J), a10 = e(I+1, J), a01 = e(I, J+1), a11 = e(I+1, J+1) with
// I = i >> 1, J = j >> 1; ox, oy = i & 1, j & 1.
template <typename T>
__device__ __forceinline__ T prolong_combine(T a00, T a10, T a01, T a11, int ox, int oy) {
  // selects rather than branches: neighbouring lanes differ in ox
  const T s0 = ox ? (T)0.5 * (a00 + a10) : a00;
  const T s1 = ox ? (T)0.5 * (a01 + a11) : a01;
  return oy ? (T)0.5 * (s0 + s1) : s0;
}

// Bilinear interpolation of the coarse correction at fine node (i, j) (row
// pitch pitchc).  At a Dirichlet boundary node it reads only stored coarse
// boundary zeros.
template <typename T>
__device__ __forceinline__ T prolong_value(const T* __restrict__ xc, int pitchc, int nyc, int py, int i, int j) {
  const int I = i >> 1, J = j >> 1;
  const int ox = i & 1, oy = j & 1;
  const T* r0 = xc + (size_t)J * pitchc;
  if (!oy) return prolong_combine(r0[I], ox ? r0[I + 1] : (T)0, (T)0, (T)0, ox, 0);
  const int J1 = (py && J + 1 == nyc) ? 0 : J + 1;
  const T* r1 = xc + (size_t)J1 * pitchc;
  return prolong_combine(r0[I], ox ? r0[I + 1] : (T)0, r1[I], ox ? r1[I + 1] : (T)0, ox, 1);
}

// The same from a coarse level held in LDS.
template <typename T>
__device__ __forceinline__ T prolong_value(const MG_LDS T* xc, int pitchc, int nyc, int py, int i, int j) {
  const int I = i >> 1, J = j >> 1;
  const int ox = i & 1, oy = j & 1;
  const MG_LDS T* r0 = xc + J * pitchc;
  if (!oy) return prolong_combine(r0[I], ox ? r0[I + 1] : (T)0, (T)0, (T)0, ox, 0);
  const int J1 = (py && J + 1 == nyc) ? 0 : J + 1;
  const MG_LDS T* r1 = xc + J1 * pitchc;
  return prolong_combine(r0[I], ox ? r0[I + 1] : (T)0, r1[I], ox ? r1[I + 1] : (T)0, ox, 1);
}

// Fine value plus the prolonged correction p, weighted by the level's
// adaptive omega_l when it has one (w = 1 adds p itself).
template <typename T>
__device__ __forceinline__ T add_correction(T t, T p, bool weighted, T w) {
  return weighted ? t + w * p : t + p;
}

// The prolonged coarse correction P e around fine node (i, j) as an x
// accessor (rows jm, j, jp already wrapped); P is a global or LDS pointer.
template <typename T, typename P>
struct PX {
  P xc;
  int pitchc, nyc, py, i, jm, j, jp;
  __device__ __forceinline__ T at(int di, int dj) const {
    return prolong_value(xc, pitchc, nyc, py, i + di, dj < 0 ? jm : (dj > 0 ? jp : j));
  }
};

// The two sums of the energy-minimising coarse-correction weight at node p
// (adaptive omega_l of "The Multigrid Technique"): s1 += d_p (P e)_p with d
// = b - A x, s2 += (A P e)_p (P e)_p; omega_l = s1 / s2 over the level.
template <int K = KDYN, typename T, typename XA, typename PA>
__device__ __forceinline__ void energy_terms(const Level<T>& L, const Cf<T>& a, const XA& x, T bp, const PA& pe,
                                             double& s1, double& s2) {
  const Nbr<T> vp = gather<K>(L, pe, true);
  const T d = defect_v<K>(L, a, gather<K>(L, x, true), bp);
  const T ape = -defect_v<K>(L, a, vp, (T)0);
  s1 += (double)d * (double)vp.c;
  s2 += (double)ape * (double)vp.c;
}

}  // namespace mg
