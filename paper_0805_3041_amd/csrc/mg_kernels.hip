// HIP kernels of the multigrid cycle for gfx950 (CDNA4, wave64).
//
// Launch convention: blockIdx.z selects the problem slot; `Ls` points at the
// level descriptor of that slot for the level the op acts on (Ls[slot]).  A
// kernel returns at once when its problem's solve is finished (st->done),
// which lets the host queue many cycles without waiting for the stopping test.
#include "mg_kernels.h"

namespace mg {

constexpr int NT = 256;  // threads per workgroup of the per-op kernels

// --------------------------------------------------------------------------- node sets

// Nodes of colour c (ncol = 2: (i + j) mod 2 == c; ncol = 4: i mod 2 == c & 1 and
// j mod 2 == c >> 1) are enumerated as (row r, slot k) with nk slots per row.
template <typename T>
struct ColourSet {
  int nk, nrows, j0, jstep;
  __device__ ColourSet(const Level<T>& L, int c, int ncol) {
    nk = (L.nx - 1) / 2 + 1;
    const int lo = row_lo(L), hi = row_hi(L);
    if (ncol == 2) {
      j0 = lo;
      jstep = 1;
      nrows = hi - lo + 1;
    } else {
      const int par = c >> 1;
      j0 = lo + ((lo & 1) != par ? 1 : 0);
      jstep = 2;
      nrows = j0 > hi ? 0 : (hi - j0) / 2 + 1;
    }
  }
  __device__ int count() const { return nk * nrows; }
  // returns false when the slot falls outside [1, nx - 2]
  __device__ bool node(const Level<T>& L, int c, int ncol, int idx, int& i, int& j) const {
    const int r = idx / nk;
    const int k = idx - r * nk;
    j = j0 + r * jstep;
    const int par = ncol == 2 ? ((c + j) & 1) : (c & 1);
    i = 2 * k + par;
    return i >= 1 && i <= L.nx - 2;
  }
};

// --------------------------------------------------------------------------- op bodies
// Each body processes the op's nodes idx = tid, tid + nth, ...

// CELLS: whether the kernel can run a finest level that forms its couplings
// from per-cell coefficients (false in the coarse-level interpreter).
template <typename T, bool CELLS = true>
__device__ void body_colour(const Level<T>& L, int c, int ncol, T omega, int tid, int nth) {
  ColourSet<T> S(L, c, ncol);
  const int n = S.count();
  for (int idx = tid; idx < n; idx += nth) {
    int i, j;
    if (!S.node(L, c, ncol, idx, i, j)) continue;
    const int jm = wrap_dn(j, L.ny, L.py), jp = wrap_up(j, L.ny, L.py);
    const size_t p = (size_t)j * L.pitch + i;
    L.x[p] = sor_v(gs_value<CELLS>(L, L.x, L.b, i, j, jm, jp), L.x + p, omega);
  }
}

template <typename T, bool CELLS = true>
__device__ void body_jacobi(const Level<T>& L, int dir, T omega, int tid, int nth) {
  const T* src = dir == 0 ? L.x : L.t;
  T* dst = dir == 0 ? L.t : L.x;
  const int lo = row_lo(L), nr = row_hi(L) - lo + 1, ni = L.nx - 2;
  const int n = nr * ni;
  for (int idx = tid; idx < n; idx += nth) {
    const int r = idx / ni;
    const int i = idx - r * ni + 1;
    const int j = lo + r;
    const int jm = wrap_dn(j, L.ny, L.py), jp = wrap_up(j, L.ny, L.py);
    dst[(size_t)j * L.pitch + i] = jacobi_value<CELLS>(L, src, L.b, i, j, jm, jp, omega);
  }
}

template <typename T>
__device__ void body_copy(const Level<T>& L, int tid, int nth) {
  const int lo = row_lo(L), nr = row_hi(L) - lo + 1, ni = L.nx - 2;
  const int n = nr * ni;
  for (int idx = tid; idx < n; idx += nth) {
    const int r = idx / ni;
    const size_t p = (size_t)(lo + r) * L.pitch + (idx - r * ni + 1);
    L.x[p] = L.t[p];
  }
}

template <typename T, bool CELLS = true>
__device__ void body_dr(const Level<T>& F, const Level<T>& C, int tid, int nth) {
  const int lo = row_lo(C), nr = row_hi(C) - lo + 1, ni = C.nx - 2;
  const int n = nr * ni;
  for (int idx = tid; idx < n; idx += nth) {
    const int r = idx / ni;
    const int I = idx - r * ni + 1;
    const int J = lo + r;
    const size_t p = (size_t)J * C.pitch + I;
    C.b[p] = restrict_defect<CELLS>(F, F.x, F.b, I, J);
    C.x[p] = (T)0;
  }
}

// x += P e (weighted: x += w P e, the adaptive omega_l).
template <typename T>
__device__ void body_prolong(const Level<T>& F, const Level<T>& C, int tid, int nth, bool weighted, T w) {
  const int lo = row_lo(F), nr = row_hi(F) - lo + 1, ni = F.nx - 2;
  const int n = nr * ni;
  for (int idx = tid; idx < n; idx += nth) {
    const int r = idx / ni;
    const int i = idx - r * ni + 1;
    const int j = lo + r;
    T* xp = F.x + (size_t)j * F.pitch + i;
    *xp = add_correction(*xp, prolong_value(C.x, C.pitch, C.ny, C.py, i, j), weighted, w);
  }
}

// Per-thread sums of the adaptive omega_l over the unknowns of F (x from a
// global array xs: F.x, or F.t after a fused pre-pass), the coarse
// correction from C.x.
template <int K, bool CELLS, typename T>
__device__ void body_energy(const Level<T>& F, const T* __restrict__ xs, const Level<T>& C, int tid, int nth,
                            double& s1, double& s2) {
  const int lo = row_lo(F), nr = row_hi(F) - lo + 1, ni = F.nx - 2;
  const int n = nr * ni;
  for (int idx = tid; idx < n; idx += nth) {
    const int r = idx / ni;
    const int i = idx - r * ni + 1;
    const int j = lo + r;
    const int jm = wrap_dn(j, F.ny, F.py), jp = wrap_up(j, F.ny, F.py);
    energy_terms<K>(F, coefs<K, CELLS>(F, i, j, jm), gx(xs, F.pitch, i, j, jm, jp), F.b[(size_t)j * F.pitch + i],
                    PX<T, const T*>{C.x, C.pitch, C.ny, C.py, i, jm, j, jp}, s1, s2);
  }
}

// Exact solve on the coarsest level: x = Ainv b with the inverse of the
// coarsest operator (n x n, row-major, unknowns numbered row by row),
// accumulated in FP64 in a fixed order.  One dot product per unknown, so no
// barrier inside the op.
template <typename T>
__device__ void body_coarse(const Level<T>& L, const double* __restrict__ Ainv, int n, int tid, int nth) {
  const int lo = row_lo(L), ni = L.nx - 2;
  for (int r = tid; r < n; r += nth) {
    const double* row = Ainv + (size_t)r * n;
    double s = 0.0;
    int i = 1, j = lo;
    for (int k = 0; k < n; ++k) {
      s = fma(row[k], (double)L.b[(size_t)j * L.pitch + i], s);
      if (++i > ni) {
        i = 1;
        ++j;
      }
    }
    const int rr = r / ni;
    L.x[(size_t)(lo + rr) * L.pitch + (r - rr * ni + 1)] = (T)s;
  }
}

// The same solve on an LDS-resident coarsest level (row pitch nx) with the
// inverse in LDS (coarsest grids of at most COARSE_LDS_MAX unknowns): the
// same products in the same order.
constexpr int COARSE_LDS_MAX = 16;
template <typename T>
__device__ void lds_coarse(const Level<T>& L, MG_LDS T* x, const MG_LDS T* b, const MG_LDS double* Ainv, int n,
                           int tid) {
  const int lo = row_lo(L), ni = L.nx - 2;
  for (int r = tid; r < n; r += SUB_NT) {
    const MG_LDS double* row = Ainv + r * n;
    double s = 0.0;
    int i = 1, j = lo;
    for (int k = 0; k < n; ++k) {
      s = fma(row[k], (double)b[j * L.nx + i], s);
      if (++i > ni) {
        i = 1;
        ++j;
      }
    }
    const int rr = r / ni;
    x[(lo + rr) * L.nx + (r - rr * ni + 1)] = (T)s;
  }
}

// --------------------------------------------------------------------------- per-op kernels

template <typename T>
__global__ void __launch_bounds__(NT) k_colour(const Level<T>* __restrict__ Ls, int c, int ncol, T omega) {
  const Level<T> L = Ls[blockIdx.z];
  if (L.st->done) return;
  body_colour(L, c, ncol, omega, blockIdx.x * NT + threadIdx.x, gridDim.x * NT);
}

template <typename T>
__global__ void __launch_bounds__(NT) k_jacobi(const Level<T>* __restrict__ Ls, int dir, T omega) {
  const Level<T> L = Ls[blockIdx.z];
  if (L.st->done) return;
  body_jacobi(L, dir, omega, blockIdx.x * NT + threadIdx.x, gridDim.x * NT);
}

template <typename T>
__global__ void __launch_bounds__(NT) k_copy(const Level<T>* __restrict__ Ls) {
  const Level<T> L = Ls[blockIdx.z];
  if (L.st->done) return;
  body_copy(L, blockIdx.x * NT + threadIdx.x, gridDim.x * NT);
}

template <typename T>
__global__ void __launch_bounds__(NT) k_dr(const Level<T>* __restrict__ Fs, const Level<T>* __restrict__ Cs) {
  const Level<T> F = Fs[blockIdx.z];
  if (F.st->done) return;
  const Level<T> C = Cs[blockIdx.z];
  body_dr(F, C, blockIdx.x * NT + threadIdx.x, gridDim.x * NT);
}

template <typename T>
__global__ void __launch_bounds__(NT) k_prolong(const Level<T>* __restrict__ Fs, const Level<T>* __restrict__ Cs,
                                                int weighted) {
  const Level<T> F = Fs[blockIdx.z];
  if (F.st->done) return;
  const Level<T> C = Cs[blockIdx.z];
  body_prolong(F, C, blockIdx.x * NT + threadIdx.x, gridDim.x * NT, weighted != 0, weighted ? *F.wl : (T)1);
}

__device__ __forceinline__ double block_sum(double v, double* sh);

// Adaptive omega_l of level F: per-workgroup partial sums s1, s2 of
// energy_terms into the slot's partial buffer (two per workgroup); x from
// F.t when src_t (after a fused pre-pass), else from F.x.
template <typename T, int K>
__global__ void __launch_bounds__(NT) k_energy(const Level<T>* __restrict__ Fs, const Level<T>* __restrict__ Cs,
                                               int src_t) {
  __shared__ double sh[NT / 64];
  const Level<T> F = Fs[blockIdx.z];
  SolveState* st = F.st;
  if (st->done) return;
  const Level<T> C = Cs[blockIdx.z];
  double s1 = 0.0, s2 = 0.0;
  body_energy<K, true>(F, src_t ? F.t : F.x, C, blockIdx.x * NT + threadIdx.x, gridDim.x * NT, s1, s2);
  const double p1 = block_sum(s1, sh);
  const double p2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    st->partial[2 * blockIdx.x] = p1;
    st->partial[2 * blockIdx.x + 1] = p2;
  }
}

// omega_l = s1 / s2 from the partial sums (fixed order), 1 when the
// prolonged correction has no energy.
template <typename T>
__global__ void __launch_bounds__(NT) k_energy_finish(const Level<T>* __restrict__ Fs, int nblocks) {
  __shared__ double sh[NT / 64];
  const Level<T> F = Fs[blockIdx.z];
  SolveState* st = F.st;
  if (st->done) return;
  double v1 = 0.0, v2 = 0.0;
  for (int k = threadIdx.x; k < nblocks; k += NT) {
    v1 += st->partial[2 * k];
    v2 += st->partial[2 * k + 1];
  }
  const double s1 = block_sum(v1, sh);
  const double s2 = block_sum(v2, sh);
  if (threadIdx.x == 0) *F.wl = (T)(s2 != 0.0 ? s1 / s2 : 1.0);
}

template <typename T>
__global__ void __launch_bounds__(NT) k_coarse(const Level<T>* __restrict__ Ls, const double* const* __restrict__ chol,
                                               int n) {
  const Level<T> L = Ls[blockIdx.z];
  if (L.st->done) return;
  body_coarse(L, chol[blockIdx.z], n, threadIdx.x, NT);
}

// --------------------------------------------------------------------------- line smoothers
// Lines along x are the rows j of unknowns (n-th node i = 1 + n), lines along
// y the columns i (n-th node j = 1 + n; Dirichlet in y only).  The tridiagonal
// part of A on a line couples node n with n - 1 (a), itself (d) and n + 1 (c);
// its Thomas factors c_n / den_n and 1 / den_n (den_n = d_n - a_n c_{n-1} /
// den_{n-1}) are formed once per level at setup.  One thread solves one line.

constexpr int LT = 64;  // threads (lines) per workgroup of the line kernels

__device__ __forceinline__ void line_node(int dir, int line, int n, int& i, int& j) {
  if (dir == 0) {
    i = 1 + n;
    j = line;
  } else {
    i = line;
    j = 1 + n;
  }
}

// Line couplings of node (i, j): a (previous node on the line), d, c (next).
template <int K, typename T>
__device__ __forceinline__ void line_coefs(const Level<T>& L, int dir, const Cf<T>& cf, T& a, T& d, T& c) {
  if (is5<K>(L)) {
    const T o = dir == 0 ? -L.cx : -L.cy;
    a = o;
    c = o;
    d = L.dg;
  } else {
    a = dir == 0 ? cf.Ew : cf.Ns;
    c = dir == 0 ? cf.Ep : cf.Np;
    d = cf.C;
  }
}

// Sum over the couplings of node p to nodes off its line, a_pq x_q.
template <int K, typename T>
__device__ __forceinline__ T off_line(const Level<T>& L, int dir, const Cf<T>& a, const Nbr<T>& v) {
  if (is5<K>(L)) return dir == 0 ? -L.cy * (v.s + v.n) : -L.cx * (v.w + v.e);
  T s;
  if (dir == 0) {
    s = a.Np * v.n;
    s = fma(a.Ns, v.s, s);
  } else {
    s = a.Ep * v.e;
    s = fma(a.Ew, v.w, s);
  }
  s = fma(a.NEp, v.ne, s);
  s = fma(a.NEsw, v.sw, s);
  s = fma(a.NWp, v.nw, s);
  s = fma(a.NWse, v.se, s);
  return s;
}

// Line `t` of a launch: every line (Jacobi) or every other line of parity
// `colour` (Gauss-Seidel); -1 past the last.
template <typename T>
__device__ __forceinline__ int line_of(const Level<T>& L, int dir, bool all, int colour, int t) {
  const int lo = dir == 0 ? row_lo(L) : 1, hi = dir == 0 ? row_hi(L) : L.nx - 2;
  const int line = all ? lo + t : lo + (((lo & 1) != colour) ? 1 : 0) + 2 * t;
  return line <= hi ? line : -1;
}

template <typename T, int K>
__global__ void __launch_bounds__(LT) k_line_factor(Level<T> L, int dir) {
  const int line = line_of(L, dir, true, 0, blockIdx.x * LT + threadIdx.x);
  if (line < 0) return;
  const int m = dir == 0 ? L.nx - 2 : L.ny - 2;
  T* cp = L.lcp[dir];
  T* id = L.lid[dir];
  T cprev = (T)0;
  for (int n = 0; n < m; ++n) {
    int i, j;
    line_node(dir, line, n, i, j);
    const Cf<T> cf = coefs<K>(L, i, j, wrap_dn(j, L.ny, L.py));
    T a, d, c;
    line_coefs<K>(L, dir, cf, a, d, c);
    const T inv = (T)1 / (d - a * cprev);
    cprev = c * inv;
    const size_t q = (size_t)j * L.pitch + i;
    cp[q] = cprev;
    id[q] = inv;
  }
}

// One line-smoothing op (arg: see line_arg).  Gauss-Seidel: x on the lines
// of one colour <- exact solution of their tridiagonal systems with the
// off-line couplings on the right-hand side (lines of one colour do not
// couple).  Jacobi (TRI): dst = src + omega T^-1 (b - A src).
template <typename T, int K, bool CELLS = true>
__device__ void line_thomas(const Level<T>& L, int arg, T omega, int t) {
  const int dir = arg & 1, sel = arg >> 2;
  const bool jac = (arg >> 1) & 1;
  const int line = line_of(L, dir, jac, sel, t);
  if (line < 0) return;
  const T* src = (jac && sel) ? L.t : L.x;
  T* dst = jac ? (sel ? L.x : L.t) : L.x;
  const int m = dir == 0 ? L.nx - 2 : L.ny - 2;
  const T* cp = L.lcp[dir];
  const T* id = L.lid[dir];
  T* rp = L.lr;
  // the loads of a node do not depend on the running recurrence: unrolled so
  // that several nodes' loads are in flight at once
  T prev = (T)0;
#pragma unroll 8
  for (int n = 0; n < m; ++n) {
    int i, j;
    line_node(dir, line, n, i, j);
    const int jm = wrap_dn(j, L.ny, L.py), jp = wrap_up(j, L.ny, L.py);
    const size_t q = (size_t)j * L.pitch + i;
    const GX<T> g{src + (size_t)jm * L.pitch + i, src + q, src + (size_t)jp * L.pitch + i};
    const Cf<T> cf = coefs<K>(L, i, j, jm);
    T a, d, c;
    line_coefs<K>(L, dir, cf, a, d, c);
    const T r = jac ? defect_v<K>(L, cf, gather<K>(L, g, true), L.b[q])
                    : L.b[q] - off_line<K>(L, dir, cf, gather<K>(L, g, false));
    prev = (r - a * prev) * id[q];
    rp[q] = prev;
  }
  T u = (T)0;
#pragma unroll 8
  for (int n = m - 1; n >= 0; --n) {
    int i, j;
    line_node(dir, line, n, i, j);
    const size_t q = (size_t)j * L.pitch + i;
    u = rp[q] - cp[q] * u;
    dst[q] = jac ? src[q] + omega * u : u;
  }
}

template <typename T, int K>
__global__ void __launch_bounds__(LT) k_line(const Level<T>* __restrict__ Ls, int arg, T omega) {
  const Level<T> L = Ls[blockIdx.z];
  if (L.st->done) return;
  line_thomas<T, K>(L, arg, omega, blockIdx.x * LT + threadIdx.x);
}

// The same op by cyclic reduction in LDS: one workgroup per line.  The
// line's tridiagonal system (a, d, c and the right-hand side of the Jacobi or
// Gauss-Seidel form above) is loaded into LDS; forward reduction eliminates,
// level by level, the couplings of the equations at (1-based) multiples of
// 2s to their neighbours at distance s; the one equation left is solved and
// back substitution recovers the rest, one barrier per level.  Every update
// of a level reads equations no update of that level writes, so all arrays
// are reduced in place.
constexpr int LCR_NT = 256;                    // threads per line
constexpr size_t LCR_LDS_MAX = 140 * 1024;     // lines with 4 m values up to this size use this kernel

template <typename T, int K>
__global__ void __launch_bounds__(LCR_NT) k_line_cr(const Level<T>* __restrict__ Ls, int arg, T omega) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Level<T> L = Ls[blockIdx.z];
  if (L.st->done) return;
  const int dir = arg & 1, sel = arg >> 2;
  const bool jac = (arg >> 1) & 1;
  const int line = line_of(L, dir, jac, sel, blockIdx.x);
  if (line < 0) return;  // uniform over the workgroup
  const int tid = threadIdx.x;
  const int m = dir == 0 ? L.nx - 2 : L.ny - 2;
  MG_LDS T* A = lds_cast<T>(smem_raw);
  MG_LDS T* D = A + m;
  MG_LDS T* C = D + m;
  MG_LDS T* R = C + m;
  const T* src = (jac && sel) ? L.t : L.x;
  T* dst = jac ? (sel ? L.x : L.t) : L.x;
  for (int n = tid; n < m; n += LCR_NT) {
    int i, j;
    line_node(dir, line, n, i, j);
    const int jm = wrap_dn(j, L.ny, L.py), jp = wrap_up(j, L.ny, L.py);
    const size_t q = (size_t)j * L.pitch + i;
    const GX<T> g{src + (size_t)jm * L.pitch + i, src + q, src + (size_t)jp * L.pitch + i};
    const Cf<T> cf = coefs<K>(L, i, j, jm);
    T a, d, c;
    line_coefs<K>(L, dir, cf, a, d, c);
    A[n] = n == 0 ? (T)0 : a;          // the line's end nodes couple to boundary values (zero)
    C[n] = n == m - 1 ? (T)0 : c;
    D[n] = d;
    R[n] = jac ? defect_v<K>(L, cf, gather<K>(L, g, true), L.b[q])
               : L.b[q] - off_line<K>(L, dir, cf, gather<K>(L, g, false));
  }
  __syncthreads();
  int s = 1;
  for (; 2 * s <= m; s *= 2) {
    for (int t = tid + 1; 2 * s * t <= m; t += LCR_NT) {
      const int p = 2 * s * t - 1, pl = p - s, pr = p + s;  // 0-based; pl >= 0
      const T al = -A[p] / D[pl];
      T nd = D[p] + al * C[pl];
      T nr = R[p] + al * R[pl];
      T nc = (T)0;
      if (pr < m) {
        const T ga = -C[p] / D[pr];
        nd += ga * A[pr];
        nr += ga * R[pr];
        nc = ga * C[pr];
      }
      A[p] = al * A[pl];
      C[p] = nc;
      D[p] = nd;
      R[p] = nr;
    }
    __syncthreads();
  }
  if (tid == 0) R[s - 1] = R[s - 1] / D[s - 1];  // the equation at s couples to nothing
  __syncthreads();
  for (s >>= 1; s >= 1; s >>= 1) {
    for (int t = tid; (2 * t + 1) * s <= m; t += LCR_NT) {
      const int p = (2 * t + 1) * s - 1, pl = p - s, pr = p + s;
      T v = R[p];
      if (pl >= 0) v -= A[p] * R[pl];
      if (pr < m) v -= C[p] * R[pr];
      R[p] = v / D[p];
    }
    __syncthreads();
  }
  for (int n = tid; n < m; n += LCR_NT) {
    int i, j;
    line_node(dir, line, n, i, j);
    const size_t q = (size_t)j * L.pitch + i;
    dst[q] = jac ? src[q] + omega * R[n] : R[n];
  }
}

// The same op for lines along y (columns, strided in memory) by segments:
// a workgroup takes LY_LINES neighbouring lines of the op and LY_SEG
// threads per line.  Phase 0 reads the lines' rows (consecutive threads on
// neighbouring lines of one row, so a row's values share cache lines) into
// LDS as a, d, c and the right-hand side.  A line's nodes are cut by
// separator nodes every B-th node into LY_SEG segments; phase 1: thread k
// eliminates segment k forward, for the right-hand side and for the
// couplings to its two separators (f: left, g: right), keeping in LDS the
// values its back substitution needs, and forms the segment's end values of
// the three solutions (first node by the running product of -c'_n, last
// node directly).  Phase 2 substitutes them into the separators' own
// equations, a tridiagonal system of LY_SEG - 1 unknowns per line, solved by
// parallel cyclic reduction in the line's wavefront.  Phase 3 substitutes
// the separator values back into every segment; phase 4 writes the rows.
// The result is the exact solution of the same systems as k_line_cr, up to
// rounding.
constexpr int LY_SEG = 64;   // segments, and threads, per line (one wavefront)
constexpr int LY_LINES = 4;  // lines per workgroup
constexpr int LY_NT = LY_SEG * LY_LINES;
constexpr int LY_MIN = 2 * LY_SEG;  // shorter lines use k_line_cr

// LDS index of node n of line li (one pad per 32 nodes: segment threads
// reading their n-th nodes at stride B hit distinct banks for B = 16, 32).
__device__ __forceinline__ int ly_at(int li, int n, int mp) { return li * mp + n + (n >> 5); }

template <typename T, int K>
__global__ void __launch_bounds__(LY_NT) k_line_y(const Level<T>* __restrict__ Ls, int arg, T omega) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ T ends[LY_LINES][6][LY_SEG];  // per segment: y, f, g at its first node, then at its last
  __shared__ T xsep[LY_LINES][LY_SEG + 1];  // separator values, [0] and [nseg] zero
  const Level<T> L = Ls[blockIdx.z];
  if (gridDim.z > 1) {
    if (L.st->done) return;
  }
  const int sel = arg >> 2;
  const bool jac = (arg >> 1) & 1;
  const int tid = threadIdx.x;
  const int m = L.ny - 2;
  const int mp = m + (m >> 5) + 1;
  MG_LDS T* A = lds_cast<T>(smem_raw);
  MG_LDS T* D = A + LY_LINES * mp;
  MG_LDS T* C = D + LY_LINES * mp;
  MG_LDS T* R = C + LY_LINES * mp;
  const T* src = (jac && sel) ? L.t : L.x;
  T* dst = jac ? (sel ? L.x : L.t) : L.x;
  const int line0 = blockIdx.x * LY_LINES;

  // phase 0: the lines' systems, row by row (a thread's rows of lines up to
  // 1024 unknowns in one batch of loads)
  constexpr int UB = 16;
  for (int idx0 = tid; idx0 < LY_LINES * m; idx0 += UB * LY_NT) {
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int idx = idx0 + u * LY_NT;
      const int li = idx % LY_LINES, n = idx / LY_LINES;
      const int line = idx < LY_LINES * m ? line_of(L, 1, jac, sel, line0 + li) : -1;
      if (line < 0) continue;
      int i, j;
      line_node(1, line, n, i, j);
      const int jm = wrap_dn(j, L.ny, L.py), jp = wrap_up(j, L.ny, L.py);
      const size_t q = (size_t)j * L.pitch + i;
      const GX<T> g{src + (size_t)jm * L.pitch + i, src + q, src + (size_t)jp * L.pitch + i};
      const Cf<T> cf = coefs<K>(L, i, j, jm);
      T a, d, c;
      line_coefs<K>(L, 1, cf, a, d, c);
      const int at = ly_at(li, n, mp);
      A[at] = n == 0 ? (T)0 : a;
      C[at] = n == m - 1 ? (T)0 : c;
      D[at] = d;
      R[at] = jac ? defect_v<K>(L, cf, gather<K>(L, g, true), L.b[q])
                  : L.b[q] - off_line<K>(L, 1, cf, gather<K>(L, g, false));
    }
  }
  const int done = L.st->done;
  __syncthreads();
  if (done) return;

  // segments: k < nseg; segment k is nodes [k B, e_k], separator k + 1 at
  // node (k + 1) B - 1 (k < nseg - 1); the last segment ends at m - 1
  const int li = tid / LY_SEG, k = tid % LY_SEG;
  const bool live = line_of(L, 1, jac, sel, line0 + li) >= 0;
  const int nseg = min(LY_SEG, (m + 1) / 2);
  const int B = (m + 1) / nseg;
  const int s0 = k * B, e0 = k == nseg - 1 ? m - 1 : (k + 1) * B - 2;
  const bool seg = live && k < nseg;

  // phase 1: forward elimination of the segment, in place: C <- c'_n, R <- y'_n, A <- f'_n;
  // the segment moves through registers in chunks of LY_CH nodes (one LDS
  // round trip per chunk, not per node)
  constexpr int LY_CH = 16;
  if (seg) {
    T cpp = (T)0, ypp = (T)0, fpp = (T)0, P = (T)1, sy = (T)0, sf = (T)0, gl = (T)0, sg = (T)0;
    T yl = (T)0, fl = (T)0;
    for (int c0 = s0; c0 <= e0; c0 += LY_CH) {
      T a[LY_CH], d[LY_CH], c[LY_CH], r[LY_CH];
#pragma unroll
      for (int u = 0; u < LY_CH; ++u)
        if (c0 + u <= e0) {
          const int at = ly_at(li, c0 + u, mp);
          a[u] = A[at];
          d[u] = D[at];
          c[u] = C[at];
          r[u] = R[at];
        }
#pragma unroll
      for (int u = 0; u < LY_CH; ++u) {
        const int n = c0 + u;
        if (n > e0) continue;
        const T inv = (T)1 / (d[u] - a[u] * cpp);
        const T cp = c[u] * inv;
        const T yp = (r[u] - a[u] * ypp) * inv;
        const T fp = (n == s0 ? -a[u] : -(a[u] * fpp)) * inv;
        c[u] = cp;
        r[u] = yp;
        a[u] = fp;
        sy += P * yp;
        sf += P * fp;
        if (n == e0) {
          yl = yp;
          fl = fp;
          gl = k < nseg - 1 ? -cp : (T)0;
          sg = P * gl;
        }
        P *= -cp;
        cpp = cp;
        ypp = yp;
        fpp = fp;
      }
#pragma unroll
      for (int u = 0; u < LY_CH; ++u)
        if (c0 + u <= e0) {
          const int at = ly_at(li, c0 + u, mp);
          A[at] = a[u];
          C[at] = c[u];
          R[at] = r[u];
        }
    }
    ends[li][0][k] = sy;
    ends[li][1][k] = sf;
    ends[li][2][k] = sg;
    ends[li][3][k] = yl;
    ends[li][4][k] = fl;
    ends[li][5][k] = gl;
  }
  __syncthreads();

  // phase 2: separator equations (thread k holds separator k, 1 <= k < nseg),
  // parallel cyclic reduction within the line's wavefront
  {
    const bool own = live && k >= 1 && k < nseg;
    T lo = (T)0, di = (T)1, up = (T)0, rh = (T)0;
    if (own) {
      const int at = ly_at(li, k * B - 1, mp);
      const T a = A[at], d = D[at], c = C[at], r = R[at];
      lo = a * ends[li][4][k - 1];
      di = d + a * ends[li][5][k - 1] + c * ends[li][1][k];
      up = k + 1 < nseg ? c * ends[li][2][k] : (T)0;
      rh = r - a * ends[li][3][k - 1] - c * ends[li][0][k];
      if (k == 1) lo = (T)0;  // segment 0 has no left separator (its f is zero)
    }
    for (int h = 1; h < nseg; h *= 2) {
      T lo_m = __shfl_up(lo, h, LY_SEG), di_m = __shfl_up(di, h, LY_SEG), up_m = __shfl_up(up, h, LY_SEG),
        rh_m = __shfl_up(rh, h, LY_SEG);
      T lo_p = __shfl_down(lo, h, LY_SEG), di_p = __shfl_down(di, h, LY_SEG), up_p = __shfl_down(up, h, LY_SEG),
        rh_p = __shfl_down(rh, h, LY_SEG);
      if (k - h < 1) {  // no equation at k - h: identity
        lo_m = (T)0;
        di_m = (T)1;
        up_m = (T)0;
        rh_m = (T)0;
      }
      if (k + h >= nseg) {
        lo_p = (T)0;
        di_p = (T)1;
        up_p = (T)0;
        rh_p = (T)0;
      }
      const T al = -lo / di_m, ga = -up / di_p;
      const T ndi = di + al * up_m + ga * lo_p;
      const T nrh = rh + al * rh_m + ga * rh_p;
      lo = al * lo_m;
      up = ga * up_p;
      di = ndi;
      rh = nrh;
    }
    if (own) xsep[li][k] = rh / di;
    if (k == 0) {
      xsep[li][0] = (T)0;
      xsep[li][nseg] = (T)0;
    }
  }
  __syncthreads();

  // phase 3: back substitution of each segment with its separators' values
  // (chunks of LY_CH nodes from the segment's end)
  if (seg) {
    const T xl = xsep[li][k], xr = xsep[li][k + 1];
    T xn = (T)0;
    for (int c1 = e0; c1 >= s0; c1 -= LY_CH) {
      T a[LY_CH], c[LY_CH], r[LY_CH];
#pragma unroll
      for (int u = 0; u < LY_CH; ++u)
        if (c1 - u >= s0) {
          const int at = ly_at(li, c1 - u, mp);
          a[u] = A[at];
          c[u] = C[at];
          r[u] = R[at];
        }
#pragma unroll
      for (int u = 0; u < LY_CH; ++u) {
        const int n = c1 - u;
        if (n < s0) continue;
        T v = r[u] + a[u] * xl;
        v = n == e0 ? v + (k < nseg - 1 ? -c[u] : (T)0) * xr : v - c[u] * xn;
        r[u] = v;
        xn = v;
      }
#pragma unroll
      for (int u = 0; u < LY_CH; ++u)
        if (c1 - u >= s0) R[ly_at(li, c1 - u, mp)] = r[u];
    }
    if (k >= 1) R[ly_at(li, k * B - 1, mp)] = xsep[li][k];
  }
  __syncthreads();

  // phase 4: the lines' new values, row by row
  for (int idx = tid; idx < LY_LINES * m; idx += LY_NT) {
    const int li2 = idx % LY_LINES, n = idx / LY_LINES;
    const int line = line_of(L, 1, jac, sel, line0 + li2);
    if (line < 0) continue;
    int i, j;
    line_node(1, line, n, i, j);
    const size_t q = (size_t)j * L.pitch + i;
    const T u = R[ly_at(li2, n, mp)];
    dst[q] = jac ? src[q] + omega * u : u;
  }
}

template <typename T>
int line_count(const Level<T>& L, int dir) {
  return dir == 0 ? (L.py ? L.ny : L.ny - 2) : L.nx - 2;
}

template <typename T>
hipError_t launch_line_factor(const Level<T>& L, int dir, hipStream_t st) {
  const int nb = (line_count(L, dir) + LT - 1) / LT;
  if (L.kind == ST5)
    hipLaunchKernelGGL((k_line_factor<T, ST5>), dim3(nb), dim3(LT), 0, st, L, dir);
  else
    hipLaunchKernelGGL((k_line_factor<T, ST9>), dim3(nb), dim3(LT), 0, st, L, dir);
  return hipGetLastError();
}

template <typename T>
hipError_t prepare_line_cr() {
  for (const void* k : {(const void*)k_line_cr<T, ST5>, (const void*)k_line_cr<T, ST9>, (const void*)k_line_y<T, ST5>,
                        (const void*)k_line_y<T, ST9>}) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LCR_LDS_MAX);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_line(const Level<T>* Ls, const LevelShape& s, int arg, T omega, int kind, int nslots,
                       hipStream_t st) {
  const int dir = arg & 1;
  const bool jac = (arg >> 1) & 1;
  int lines = dir == 0 ? s.nrows : s.nx - 2;
  if (!jac) lines = (lines + 1) / 2;
  const int m = dir == 0 ? s.nx - 2 : s.ny - 2;
  const size_t ylds = 4 * (size_t)LY_LINES * (m + (m >> 5) + 1) * sizeof(T);
  if (dir == 1 && m >= LY_MIN && ylds <= LCR_LDS_MAX) {
    const dim3 grid((lines + LY_LINES - 1) / LY_LINES, 1, nslots);
    if (kind == ST5)
      hipLaunchKernelGGL((k_line_y<T, ST5>), grid, dim3(LY_NT), ylds, st, Ls, arg, omega);
    else
      hipLaunchKernelGGL((k_line_y<T, ST9>), grid, dim3(LY_NT), ylds, st, Ls, arg, omega);
    return hipGetLastError();
  }
  const size_t lds = 4 * (size_t)m * sizeof(T);
  if (lds <= LCR_LDS_MAX) {
    const dim3 grid(lines, 1, nslots);
    if (kind == ST5)
      hipLaunchKernelGGL((k_line_cr<T, ST5>), grid, dim3(LCR_NT), lds, st, Ls, arg, omega);
    else
      hipLaunchKernelGGL((k_line_cr<T, ST9>), grid, dim3(LCR_NT), lds, st, Ls, arg, omega);
    return hipGetLastError();
  }
  const dim3 grid((lines + LT - 1) / LT, 1, nslots);
  if (kind == ST5)
    hipLaunchKernelGGL((k_line<T, ST5>), grid, dim3(LT), 0, st, Ls, arg, omega);
  else
    hipLaunchKernelGGL((k_line<T, ST9>), grid, dim3(LT), 0, st, Ls, arg, omega);
  return hipGetLastError();
}

// --------------------------------------------------------------------------- op bodies on LDS levels
// Levels held in LDS as dense [ny][nx] arrays (row pitch nx).  Threads map to
// (column, row group) with power-of-two column groups and 32-bit offsets, so
// the loops need no division; the node arithmetic is the shared one.

__device__ __forceinline__ int ceil_log2(int v) { return v <= 1 ? 0 : 32 - __clz(v - 1); }

template <typename T>
__device__ __forceinline__ LX3<T> lgx(const MG_LDS T* x, int nx, int i, int j, int jm, int jp) {
  return LX3<T>{x + jm * nx + i, x + j * nx + i, x + jp * nx + i};
}

// Coefficients of node (i, j) on an LDS-resident level: B1 (9-point bands
// that vary along x only) from the level's LDS copy of its bands (band k at
// bl + k nx, the same values as coefs()), otherwise the bands (the
// interpreter runs coarse levels only, which keep no cell coefficients).
template <typename T, int K, bool B1>
__device__ __forceinline__ Cf<T> sub_coefs(const Level<T>& L, const MG_LDS T* bl, int i, int j, int jm) {
  if constexpr (K == ST9 && B1) {
    const int nx = L.nx;
    const MG_LDS T* p = bl + i;
    Cf<T> c;
    c.C = p[0];
    c.Ep = p[nx];
    c.Ew = p[nx - 1];
    c.Np = p[2 * nx];
    c.Ns = c.Np;
    c.NEp = p[3 * nx];
    c.NEsw = p[3 * nx - 1];
    c.NWp = p[4 * nx];
    c.NWse = p[4 * nx + 1];
    c.D = p[BAND_D * nx];
    return c;
  } else {
    return coefs<K, false>(L, i, j, jm);
  }
}

// LDS level array around the node at p: rows below and above at offsets
// so (-nx, or +(ny-1) nx across a periodic seam) and no (+nx, or -(ny-1) nx).
template <typename T>
struct LXO {
  const MG_LDS T* p;
  int so, no;
  __device__ __forceinline__ T at(int di, int dj) const { return p[(dj < 0 ? so : (dj > 0 ? no : 0)) + di]; }
};

// Offsets of the rows below and above row j of an LDS level (periodic seam).
__device__ __forceinline__ void row_offsets(int j, int nx, int ny, int py, int& so, int& no) {
  so = (py && j == 0) ? (ny - 1) * nx : -nx;
  no = (py && j == ny - 1) ? -(ny - 1) * nx : nx;
}

// Gauss-Seidel update of colour c.  Thread -> (column slot k, row group);
// a thread's column is fixed for the op (row groups step by an even number
// of rows, so the colour's column offset is the same on all its rows), its
// rows advance by a uniform stride, and coefficients that depend on the
// column only are read once.
//
// Column i, first row j and row stride of thread `tid` for colour c.
template <typename T, int NTH = SUB_NT>
__device__ __forceinline__ void colour_plan(const Level<T>& L, int c, int ncol, int tid, int& i, int& j, int& jstep) {
  const int lo = L.py ? 0 : 1;
  const int kl = ceil_log2((L.nx - 1) >> 1);
  const int k = tid & ((1 << kl) - 1);
  const int rg = NTH >> kl;  // even: kl <= 9 for every LDS level (kl <= 5 with one wave)
  int first;
  if (ncol == 4) {
    j = lo + (((lo & 1) != (c >> 1)) ? 1 : 0) + 2 * (tid >> kl);
    jstep = 2 * rg;
    first = (c & 1) ? 1 : 2;
  } else {
    j = lo + (tid >> kl);
    jstep = rg;
    first = 1 + ((((1 + j) & 1) != c) ? 1 : 0);
  }
  i = first + 2 * k;
}

// The colour's nodes of column i on rows j, j + jstep, ... <= hi.
template <typename T, int K, bool B1>
__device__ __forceinline__ void colour_rows(const Level<T>& L, MG_LDS T* x, const MG_LDS T* b, const MG_LDS T* bl,
                                            int i, int j, int jstep, const Cf<T>& col, T omega) {
  constexpr int NB = nbatch(K);
  const int nx = L.nx, ny = L.ny, py = L.py;
  const int hi = py ? ny - 1 : ny - 2;
  const bool col_only = K == ST5 || B1;
  const int dpos = jstep * nx;
  int pos = j * nx + i;
  for (; j <= hi; j += NB * jstep, pos += NB * dpos) {
    Nbr<T> v[NB];
    Cf<T> a[NB];
    T bp[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int ju = j + u * jstep;
      if (ju > hi) continue;
      int so, no;
      row_offsets(ju, nx, ny, py, so, no);
      v[u] = gather<K>(L, LXO<T>{x + pos + u * dpos, so, no}, false);
      bp[u] = b[pos + u * dpos];
      a[u] = col_only ? col : sub_coefs<T, K, B1>(L, bl, i, ju, wrap_dn(ju, ny, py));
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (j + u * jstep <= hi) x[pos + u * dpos] = sor_v(gs_v<K>(L, a[u], v[u], bp[u]), x + pos + u * dpos, omega);
  }
}

template <typename T, int K, bool B1>
__device__ void lds_colour(const Level<T>& L, MG_LDS T* x, const MG_LDS T* b, const MG_LDS T* bl, int c, int ncol,
                           T omega, int tid) {
  int i, j, jstep;
  colour_plan(L, c, ncol, tid, i, j, jstep);
  if (i > L.nx - 2) return;
  Cf<T> col{};
  if (K == ST5 || B1) col = sub_coefs<T, K, B1>(L, bl, i, 0, 0);
  colour_rows<T, K, B1>(L, x, b, bl, i, j, jstep, col, omega);
}

template <typename T, int K, bool B1>
__device__ void lds_jacobi(const Level<T>& L, const MG_LDS T* src, MG_LDS T* dst, const MG_LDS T* b,
                           const MG_LDS T* bl, T omega, int tid) {
  constexpr int NB = nbatch(K);
  const int nx = L.nx, ny = L.ny, py = L.py;
  const int lo = py ? 0 : 1, hi = py ? ny - 1 : ny - 2;
  const int kl = ceil_log2(nx - 2);
  const int i = 1 + (tid & ((1 << kl) - 1));
  if (i > nx - 2) return;
  const bool col_only = K == ST5 || B1;
  Cf<T> col{};
  if (col_only) col = sub_coefs<T, K, B1>(L, bl, i, 0, 0);
  const int jstep = SUB_NT >> kl, dpos = jstep * nx;
  int j = lo + (tid >> kl), pos = j * nx + i;
  for (; j <= hi; j += NB * jstep, pos += NB * dpos) {
    Nbr<T> v[NB];
    Cf<T> a[NB];
    T bp[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int ju = j + u * jstep;
      if (ju > hi) continue;
      int so, no;
      row_offsets(ju, nx, ny, py, so, no);
      v[u] = gather<K>(L, LXO<T>{src + pos + u * dpos, so, no}, true);
      bp[u] = b[pos + u * dpos];
      a[u] = col_only ? col : sub_coefs<T, K, B1>(L, bl, i, ju, wrap_dn(ju, ny, py));
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (j + u * jstep <= hi) dst[pos + u * dpos] = jac_v<K>(L, a[u], v[u], bp[u], omega);
  }
}

template <typename T>
__device__ void lds_copy(const Level<T>& L, MG_LDS T* x, const MG_LDS T* t, int tid) {
  const int nx = L.nx, ny = L.ny, py = L.py;
  const int lo = py ? 0 : 1, hi = py ? ny - 1 : ny - 2;
  const int kl = ceil_log2(nx - 2);
  const int i = 1 + (tid & ((1 << kl) - 1));
  if (i > nx - 2) return;
  for (int j = lo + (tid >> kl); j <= hi; j += SUB_NT >> kl) x[j * nx + i] = t[j * nx + i];
}

template <typename T, int K, bool B1>
__device__ void lds_dr(const Level<T>& F, const MG_LDS T* xf, const MG_LDS T* bf, const MG_LDS T* bl,
                       const Level<T>& C, MG_LDS T* xc, MG_LDS T* bc, int tid) {
  const int nx = F.nx, ny = F.ny, py = F.py;
  const int lo = C.py ? 0 : 1, hi = C.py ? C.ny - 1 : C.ny - 2;
  const int kl = ceil_log2(C.nx - 2);
  const int I = 1 + (tid & ((1 << kl) - 1));
  if (I > C.nx - 2) return;
  for (int J = lo + (tid >> kl); J <= hi; J += SUB_NT >> kl) {
    const int i0 = 2 * I, j0 = 2 * J;
    const int rows[3] = {wrap_dn(j0, ny, py), j0, wrap_up(j0, ny, py)};
    T acc[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int j = rows[r];
      const int jm = wrap_dn(j, ny, py), jp = wrap_up(j, ny, py);
      const int q = j * nx;
      const T dw = defect_v<K>(F, sub_coefs<T, K, B1>(F, bl, i0 - 1, j, jm),
                               gather<K>(F, lgx(xf, nx, i0 - 1, j, jm, jp), true), bf[q + i0 - 1]);
      const T dc = defect_v<K>(F, sub_coefs<T, K, B1>(F, bl, i0, j, jm), gather<K>(F, lgx(xf, nx, i0, j, jm, jp), true),
                               bf[q + i0]);
      const T de = defect_v<K>(F, sub_coefs<T, K, B1>(F, bl, i0 + 1, j, jm),
                               gather<K>(F, lgx(xf, nx, i0 + 1, j, jm, jp), true), bf[q + i0 + 1]);
      acc[r] = fw_row(dw, dc, de);
    }
    const int pc = J * C.nx + I;
    bc[pc] = fw_combine(acc[0], acc[1], acc[2]);
    xc[pc] = (T)0;
  }
}

template <typename T>
__device__ void lds_prolong(const Level<T>& F, MG_LDS T* xf, const Level<T>& C, const MG_LDS T* xc, int tid,
                            bool weighted, T w) {
  const int nx = F.nx, ny = F.ny, py = F.py;
  const int lo = py ? 0 : 1, hi = py ? ny - 1 : ny - 2;
  const int kl = ceil_log2(nx - 2);
  const int i = 1 + (tid & ((1 << kl) - 1));
  if (i > nx - 2) return;
  const int I = i >> 1, ox = i & 1;
  for (int j = lo + (tid >> kl); j <= hi; j += SUB_NT >> kl) {
    const int J = j >> 1, oy = j & 1;
    const MG_LDS T* r0 = xc + J * C.nx + I;
    T v;
    if (!oy) {
      v = prolong_combine(r0[0], ox ? r0[1] : (T)0, (T)0, (T)0, ox, 0);
    } else {
      const int J1 = (py && J + 1 == C.ny) ? 0 : J + 1;
      const MG_LDS T* r1 = xc + J1 * C.nx + I;
      v = prolong_combine(r0[0], ox ? r0[1] : (T)0, r1[0], ox ? r1[1] : (T)0, ox, 1);
    }
    xf[j * nx + i] = add_correction(xf[j * nx + i], v, weighted, w);
  }
}

// `nsw` whole Gauss-Seidel sweeps (colours 0 .. ncol - 1 in order) as one op:
// the same node updates as nsw * ncol OP_COLOR ops, with each thread's
// columns and column coefficients found once and a workgroup barrier
// between colours (the interpreter's own barrier follows the last).  Even
// and odd colours differ in their column parity only (4 colours) or are the
// two colours (2 colours), so two coefficient sets cover every colour.
template <typename T, int K, bool B1, int NCOL>
__device__ void lds_smooth_n(const Level<T>& L, MG_LDS T* x, const MG_LDS T* b, const MG_LDS T* bl, int nsw, T omega,
                             int tid) {
  const int last = L.nx - 2;
  int ic[NCOL], jc[NCOL], js[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) colour_plan(L, c, NCOL, tid, ic[c], jc[c], js[c]);
  Cf<T> c0{}, c1{};
  if (K == ST5 || B1) {
    if (ic[0] <= last) c0 = sub_coefs<T, K, B1>(L, bl, ic[0], 0, 0);
    if (ic[1] <= last) c1 = sub_coefs<T, K, B1>(L, bl, ic[1], 0, 0);
  }
  for (int s = 0; s < nsw; ++s) {
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
      if (ic[c] <= last) colour_rows<T, K, B1>(L, x, b, bl, ic[c], jc[c], js[c], (c & 1) ? c1 : c0, omega);
      if (s + 1 < nsw || c + 1 < NCOL) __syncthreads();
    }
  }
}

// Same sweeps when no thread has more than M rows of any colour (the levels
// at the bottom of the hierarchy): each thread's nodes, their row offsets
// and right-hand sides (fixed while smoothing) are found once, so a colour
// step is the gather, the update and the store.
//
// SOLO: wavefront 0 alone owns every node (the plan over 64 threads; levels
// whose colours have at most one row per lane), and its colour steps are
// ordered by waiting for its own LDS writes instead of by workgroup
// barriers (a wavefront's LDS operations complete in issue order; the wait
// makes every store land before the next step's gathers issue).  The other
// wavefronts do not enter: nothing in here may wait on them.
template <bool SOLO>
__device__ __forceinline__ void step_sync() {
  if constexpr (SOLO) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // (keeps the compiler's order of LDS accesses)
    __builtin_amdgcn_s_waitcnt(0xc07f);                       // lgkmcnt(0): this wave's LDS stores have landed
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <typename T, int K, bool B1, int NCOL, int M, bool SOLO = false>
__device__ void lds_smooth_few(const Level<T>& L, MG_LDS T* x, const MG_LDS T* b, const MG_LDS T* bl, int nsw,
                               T omega, int tid, const Level<T>& C, const MG_LDS T* xc, int flags, T wl) {
  const int nx = L.nx, ny = L.ny, py = L.py;
  const int hi = py ? ny - 1 : ny - 2, last = nx - 2;
  constexpr bool col_only = K == ST5 || B1;
  int ic[NCOL], pos[NCOL][M], so[NCOL][M], no[NCOL][M], jr[NCOL][M];
  T bv[NCOL][M];
  bool on[NCOL][M];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) {
    int j, jstep;
    colour_plan<T, SOLO ? 64 : SUB_NT>(L, c, NCOL, tid, ic[c], j, jstep);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int jm = j + m * jstep;
      on[c][m] = ic[c] <= last && jm <= hi;
      jr[c][m] = jm;
      pos[c][m] = jm * nx + ic[c];
      so[c][m] = no[c][m] = 0;
      bv[c][m] = (T)0;
      if (on[c][m]) {
        row_offsets(jm, nx, ny, py, so[c][m], no[c][m]);
        bv[c][m] = b[pos[c][m]];
      }
    }
  }
  Cf<T> c0{}, c1{};
  if (col_only) {
    if (ic[0] <= last) c0 = sub_coefs<T, K, B1>(L, bl, ic[0], 0, 0);
    if (ic[1] <= last) c1 = sub_coefs<T, K, B1>(L, bl, ic[1], 0, 0);
  }
  if (flags & SM_PRO) {
    // the coarse-grid correction, node by node as lds_prolong forms it, on
    // the nodes this thread owns (the colours' plans cover every unknown once)
    const bool wtd = (flags & SM_WTD) != 0;
#pragma unroll
    for (int c = 0; c < NCOL; ++c)
#pragma unroll
      for (int m = 0; m < M; ++m)
        if (on[c][m]) {
          const int i = ic[c], j = jr[c][m];
          const int I = i >> 1, ox = i & 1, J = j >> 1;
          const MG_LDS T* r0 = xc + J * C.nx + I;
          T v;
          if (!(j & 1)) {
            v = prolong_combine(r0[0], ox ? r0[1] : (T)0, (T)0, (T)0, ox, 0);
          } else {
            const int J1 = (py && J + 1 == C.ny) ? 0 : J + 1;
            const MG_LDS T* r1 = xc + J1 * C.nx + I;
            v = prolong_combine(r0[0], ox ? r0[1] : (T)0, r1[0], ox ? r1[1] : (T)0, ox, 1);
          }
          x[pos[c][m]] = add_correction(x[pos[c][m]], v, wtd, wl);
        }
    step_sync<SOLO>();
  }
  for (int s = 0; s < nsw; ++s) {
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
      Nbr<T> v[M];
      Cf<T> a[M];
#pragma unroll
      for (int m = 0; m < M; ++m)
        if (on[c][m]) {
          v[m] = gather<K>(L, LXO<T>{x + pos[c][m], so[c][m], no[c][m]}, false);
          a[m] = col_only ? ((c & 1) ? c1 : c0)
                          : sub_coefs<T, K, B1>(L, bl, ic[c], jr[c][m], wrap_dn(jr[c][m], ny, py));
        }
#pragma unroll
      for (int m = 0; m < M; ++m)
        if (on[c][m]) x[pos[c][m]] = sor_v(gs_v<K>(L, a[m], v[m], bv[c][m]), x + pos[c][m], omega);
      if (s + 1 < nsw || c + 1 < NCOL) step_sync<SOLO>();
    }
  }
  if constexpr (SOLO) step_sync<true>();
}

// Rows per thread of one colour: at most ceil(rows / row stride); the
// register-resident form where that is 1 (or 2 with two colours).  The
// block's transfers (flags): SM_PRO adds the level's coarse-grid
// correction before the sweeps (the register-resident form on its own
// nodes, otherwise as its own pass), SM_DR restricts the defect into level
// + 1 after them; C and xc are level + 1 and its x in LDS.
template <typename T, int K, bool B1, int NCOL>
__device__ __forceinline__ void lds_smooth_c(const Level<T>& L, MG_LDS T* x, const MG_LDS T* b, const MG_LDS T* bl,
                                             int nsw, T omega, int tid, const Level<T>& C, MG_LDS T* xc, int flags,
                                             T wl) {
  const int kl = ceil_log2((L.nx - 1) >> 1);
  const int rstride = (NCOL == 4 ? 2 : 1) * (SUB_NT >> kl);
  const int rows = L.py ? L.ny : L.ny - 2;
  const int m = (rows + rstride - 1) / rstride;
  // one row per lane of wavefront 0 for every colour: that wave alone
  const bool solo = kl <= 5 && rows <= (NCOL == 4 ? 2 : 1) * (64 >> kl);
  if (solo) {
    if (tid < 64) lds_smooth_few<T, K, B1, NCOL, 1, true>(L, x, b, bl, nsw, omega, tid, C, xc, flags, wl);
  } else if (m <= 1) {
    lds_smooth_few<T, K, B1, NCOL, 1>(L, x, b, bl, nsw, omega, tid, C, xc, flags, wl);
  } else if (NCOL == 2 && m <= 2) {  // (two rows of four colours would spill registers)
    lds_smooth_few<T, K, B1, NCOL, 2>(L, x, b, bl, nsw, omega, tid, C, xc, flags, wl);
  } else {
    if (flags & SM_PRO) {
      lds_prolong(L, x, C, xc, tid, (flags & SM_WTD) != 0, wl);
      __syncthreads();
    }
    lds_smooth_n<T, K, B1, NCOL>(L, x, b, bl, nsw, omega, tid);
  }
  if (flags & SM_DR) {
    __syncthreads();
    lds_dr<T, K, B1>(L, x, b, bl, C, xc, xc + C.nx * C.ny, tid);
  }
}

// (9-point operators are smoothed with four colours only: setup rejects
// red-black Gauss-Seidel for them.)
template <typename T, int K, bool B1>
__device__ void lds_smooth(const Level<T>& L, MG_LDS T* x, const MG_LDS T* b, const MG_LDS T* bl, int nsw, int ncol,
                           T omega, int tid, const Level<T>& C, MG_LDS T* xc, int flags, T wl) {
  if constexpr (K == ST9) {
    lds_smooth_c<T, K, B1, 4>(L, x, b, bl, nsw, omega, tid, C, xc, flags, wl);
  } else {
    if (ncol == 4)
      lds_smooth_c<T, K, B1, 4>(L, x, b, bl, nsw, omega, tid, C, xc, flags, wl);
    else
      lds_smooth_c<T, K, B1, 2>(L, x, b, bl, nsw, omega, tid, C, xc, flags, wl);
  }
}

// Per-thread sums of the adaptive omega_l of an LDS level (threads mapped as
// in lds_copy; threads past the last column add nothing).
template <typename T, int K, bool B1>
__device__ void lds_energy(const Level<T>& F, const MG_LDS T* xf, const MG_LDS T* bf, const MG_LDS T* bl,
                           const Level<T>& C, const MG_LDS T* xc, int tid, double& s1, double& s2) {
  const int nx = F.nx, ny = F.ny, py = F.py;
  const int lo = py ? 0 : 1, hi = py ? ny - 1 : ny - 2;
  const int kl = ceil_log2(nx - 2);
  const int i = 1 + (tid & ((1 << kl) - 1));
  if (i > nx - 2) return;
  for (int j = lo + (tid >> kl); j <= hi; j += SUB_NT >> kl) {
    const int jm = wrap_dn(j, ny, py), jp = wrap_up(j, ny, py);
    energy_terms<K>(F, sub_coefs<T, K, B1>(F, bl, i, j, jm), lgx(xf, nx, i, j, jm, jp), bf[j * nx + i],
                    PX<T, const MG_LDS T*>{xc, C.nx, C.ny, C.py, i, jm, j, jp}, s1, s2);
  }
}

// Line sweep of an LDS level inside the coarse-level kernel: every line of
// the op (all lines for Jacobi, one zebra colour for Gauss-Seidel) is solved
// at once by cyclic reduction in the scratch `scr` (4 values per node of the
// swept lines), each reduction level one workgroup barrier; the arithmetic
// per equation is that of k_line_cr.  Called by every thread of the
// workgroup.
template <typename T, int K, bool B1>
__device__ void lds_line(const Level<T>& L, MG_LDS T* x, const MG_LDS T* b, MG_LDS T* t, const MG_LDS T* bl,
                         MG_LDS T* scr, int arg, T omega, int tid) {
  const int nx = L.nx, ny = L.ny, py = L.py;
  const int dir = arg & 1, sel = arg >> 2;
  const bool jac = (arg >> 1) & 1;
  const int m = dir == 0 ? nx - 2 : ny - 2;
  const int lo = dir == 0 ? (py ? 0 : 1) : 1, hi = dir == 0 ? (py ? ny - 1 : ny - 2) : nx - 2;
  const int first = jac ? lo : lo + (((lo & 1) != sel) ? 1 : 0);
  const int step = jac ? 1 : 2;
  const int nl = hi >= first ? (hi - first) / step + 1 : 0;
  const MG_LDS T* src = (jac && sel) ? t : x;
  MG_LDS T* dst = jac ? (sel ? x : t) : x;
  const int tot = nl * m;
  MG_LDS T* A = scr;
  MG_LDS T* D = A + tot;
  MG_LDS T* C = D + tot;
  MG_LDS T* R = C + tot;
  const FDiv dm(m);
  for (int idx = tid; idx < tot; idx += SUB_NT) {
    const int li = dm.q(idx), n = idx - li * m;
    int i, j;
    line_node(dir, first + step * li, n, i, j);
    const int jm = wrap_dn(j, ny, py);
    int so, no;
    row_offsets(j, nx, ny, py, so, no);
    const int p = j * nx + i;
    const Cf<T> cf = sub_coefs<T, K, B1>(L, bl, i, j, jm);
    T a, d, c;
    line_coefs<K>(L, dir, cf, a, d, c);
    A[idx] = n == 0 ? (T)0 : a;
    C[idx] = n == m - 1 ? (T)0 : c;
    D[idx] = d;
    R[idx] = jac ? defect_v<K>(L, cf, gather<K>(L, LXO<T>{src + p, so, no}, true), b[p])
                 : b[p] - off_line<K>(L, dir, cf, gather<K>(L, LXO<T>{src + p, so, no}, false));
  }
  __syncthreads();
  int s = 1;
  for (; 2 * s <= m; s *= 2) {
    const int u = m / (2 * s);  // reductions per line at this level
    const FDiv du(u);
    for (int idx = tid; idx < nl * u; idx += SUB_NT) {
      const int li = du.q(idx), base = li * m;
      const int pp = 2 * s * (idx - li * u + 1) - 1;  // position on the line (0-based)
      const int p = base + pp, pl = p - s, pr = p + s;
      const T al = -A[p] / D[pl];
      T nd = D[p] + al * C[pl];
      T nr = R[p] + al * R[pl];
      T nc = (T)0;
      if (pp + s < m) {
        const T ga = -C[p] / D[pr];
        nd += ga * A[pr];
        nr += ga * R[pr];
        nc = ga * C[pr];
      }
      A[p] = al * A[pl];
      C[p] = nc;
      D[p] = nd;
      R[p] = nr;
    }
    __syncthreads();
  }
  for (int li = tid; li < nl; li += SUB_NT) {
    const int q = li * m + s - 1;
    R[q] = R[q] / D[q];
  }
  __syncthreads();
  for (s >>= 1; s >= 1; s >>= 1) {
    const int v = (m / s + 1) / 2;  // odd multiples of s on a line
    const FDiv dv(v);
    for (int idx = tid; idx < nl * v; idx += SUB_NT) {
      const int li = dv.q(idx), base = li * m;
      const int pp = (2 * (idx - li * v) + 1) * s - 1;
      const int p = base + pp;
      T w = R[p];
      if (pp - s >= 0) w -= A[p] * R[p - s];
      if (pp + s < m) w -= C[p] * R[p + s];
      R[p] = w / D[p];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < tot; idx += SUB_NT) {
    const int li = dm.q(idx), n = idx - li * m;
    int i, j;
    line_node(dir, first + step * li, n, i, j);
    const int p = j * nx + i;
    dst[p] = jac ? src[p] + omega * R[idx] : R[idx];
  }
}

// Single-workgroup interpreter: runs ops [beg[slot], beg[slot] + cnt[slot]) of
// `prog` on the levels of its slot (levs + slot * nlev), one barrier between
// ops.  Used for every level small enough that a launch per op would cost
// more than the op itself.  The op list and the level descriptors are first
// copied to LDS so that no op waits on a global load to learn what to do.
// IN_LDS: every level from `top` down also lives in LDS (x, b and, for
// Jacobi, t as dense [ny][nx] arrays): the top level's x and b are read once
// and x written back at exit; coarser levels never leave LDS.  Bands
// (9-point operators) are read from global memory, 1-D bands from an LDS
// copy; line sweeps use a scratch after the levels.
__device__ __forceinline__ int pack_op(const DOp& o) { return o.type | (o.level << 4) | (o.arg << 12); }

template <typename T, bool IN_LDS, int K, bool B1 = false>
__global__ void __launch_bounds__(SUB_NT) k_subcycle(const Level<T>* __restrict__ levs, int nlev, int top,
                                                     const DOp* __restrict__ prog, const int* __restrict__ beg,
                                                     const int* __restrict__ cnt,
                                                     const double* const* __restrict__ chol, int ncu, T omega,
                                                     int ncol, int narr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  MG_LDS T* lds = lds_cast<T>(smem_raw);
  __shared__ int offs[MAX_LEVELS + 1];
  __shared__ int boffs[MAX_LEVELS];  // B1: LDS offset of each level's bands
  __shared__ int soff;               // LDS offset of the line-sweep scratch
  __shared__ int sops[MAX_SUB_OPS];
  __shared__ double esh[SUB_NT / 64];  // workgroup sums of OP_OMEGA
  __shared__ T wsh[MAX_LEVELS];        // adaptive omega_l per level, set by OP_OMEGA
  __shared__ double ainv_sh[COARSE_LDS_MAX * COARSE_LDS_MAX];  // small coarsest inverse
  const int slot = blockIdx.z;
  const Level<T>* Ls = levs + (size_t)slot * nlev;
  // A batched launch skips a finished problem at once; one problem reads the
  // flag with its first loads and tests it before the first op (nothing is
  // stored before that), so the preamble's loads do not wait on it.
  if (gridDim.z > 1) {
    if (Ls[0].st->done) return;
  }
  const int tid = threadIdx.x;
  const int b0 = beg[slot], nops = cnt[slot];
  const bool ops_in_lds = nops <= MAX_SUB_OPS;
  if (ops_in_lds)
    for (int k = tid; k < nops; k += SUB_NT) sops[k] = pack_op(prog[b0 + k]);
  if (IN_LDS && tid == 0) {
    int o = 0;
    for (int l = top; l < nlev; ++l) {
      offs[l] = o;
      o += narr * Ls[l].nx * Ls[l].ny;
    }
    offs[nlev] = o;
    if (B1)
      for (int l = top; l < nlev; ++l) {
        boffs[l] = o;
        o += NBANDS * Ls[l].nx;
      }
    soff = o;
  }
  const int done = Ls[0].st->done;
  __syncthreads();
  if (IN_LDS) {
    // One phase, one barrier: the top level's interior x and b and every
    // level's 1-D bands are loaded (several loads in flight per thread)
    // while every other entry of the levels is zeroed.
    const Level<T> G = Ls[top];
    const int gnx = G.nx, gny = G.ny, gn = gnx * gny;
    const int lo = row_lo(G), nr = row_hi(G) - lo + 1, ni = gnx - 2, n = nr * ni;
    MG_LDS T* xl = lds + offs[top];
    MG_LDS T* bl = xl + gn;
    constexpr int UB = 4;
    const FDiv dni(ni);
    for (int idx0 = tid; idx0 < n; idx0 += UB * SUB_NT) {
      T xv[UB], bv[UB];
      int pos[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int idx = idx0 + u * SUB_NT;
        pos[u] = -1;
        if (idx < n) {
          const int r = dni.q(idx);
          const int i = idx - r * ni + 1, j = lo + r;
          pos[u] = j * gnx + i;
          xv[u] = G.x[(size_t)j * G.pitch + i];
          bv[u] = G.b[(size_t)j * G.pitch + i];
        }
      }
#pragma unroll
      for (int u = 0; u < UB; ++u)
        if (pos[u] >= 0) {
          xl[pos[u]] = xv[u];
          bl[pos[u]] = bv[u];
        }
    }
    if (B1) {
      int nb = 0;
      for (int l = top; l < nlev; ++l) nb += NBANDS * Ls[l].nx;
      for (int e = tid; e < nb; e += SUB_NT) {
        int l = top, k = e;
        while (k >= NBANDS * Ls[l].nx) {
          k -= NBANDS * Ls[l].nx;
          ++l;
        }
        const Level<T>& Lb = Ls[l];
        const int band = k / Lb.nx, i = k - band * Lb.nx;
        lds[boffs[l] + k] = bandp(Lb, band)[i];
      }
    }
    if (ncu <= COARSE_LDS_MAX)
      for (int k = tid; k < ncu * ncu; k += SUB_NT) ainv_sh[k] = chol[slot][k];
    // zeros: the top level's boundary nodes of x and b, its t (Jacobi), and
    // every coarser level
    for (int k = tid; k < 2 * gny; k += SUB_NT) {
      const int arr = k / gny, j = k - arr * gny;
      MG_LDS T* a = xl + arr * gn + j * gnx;
      a[0] = (T)0;
      a[gnx - 1] = (T)0;
    }
    if (!G.py)
      for (int k = tid; k < 2 * gnx; k += SUB_NT) {
        const int arr = k / gnx, i = k - arr * gnx;
        MG_LDS T* a = xl + arr * gn + i;
        a[0] = (T)0;
        a[(gny - 1) * gnx] = (T)0;
      }
    const int total = offs[nlev];
    for (int k = offs[top] + 2 * gn + tid; k < total; k += SUB_NT) lds[k] = (T)0;
    __syncthreads();
  }
  if (done) return;
  for (int k = 0; k < nops; ++k) {
    // op and level descriptor through the scalar cache (uniform index)
    int type, l, arg;
    if (ops_in_lds) {
      const int w = __builtin_amdgcn_readfirstlane(sops[k]);
      type = w & 15;
      l = (w >> 4) & 255;
      arg = w >> 12;
    } else {
      const DOp o = prog[b0 + k];
      type = o.type;
      l = o.level;
      arg = o.arg;
    }
    Level<T> L = Ls[l];
    if (IN_LDS) {
      const int nl = L.nx * L.ny;
      L.x = (T*)(lds + offs[l]);  // generic view, used by the coarsest solve only
      L.b = L.x + nl;
      L.t = L.b + nl;
      L.pitch = L.nx;
    }
    if (IN_LDS) {
      MG_LDS T* xl = lds + offs[l];
      MG_LDS T* bl = xl + L.nx * L.ny;
      MG_LDS T* tl = bl + L.nx * L.ny;
      const MG_LDS T* bands = B1 ? lds + boffs[l] : nullptr;
      switch (type) {
        case OP_COLOR: lds_colour<T, K, B1>(L, xl, bl, bands, arg, ncol, omega, tid); break;
        case OP_SMOOTH: {
          const bool tr = (arg & (SM_PRO | SM_DR)) != 0;  // level + 1 exists then
          const Level<T> C = tr ? Ls[l + 1] : L;
          lds_smooth<T, K, B1>(L, xl, bl, bands, arg & SM_NSW, ncol, omega, tid, C, tr ? lds + offs[l + 1] : xl,
                               arg, tr ? wsh[l] : (T)1);
          break;
        }
        case OP_JACOBI:
          lds_jacobi<T, K, B1>(L, arg == 0 ? xl : tl, arg == 0 ? tl : xl, bl, bands, omega, tid);
          break;
        case OP_COPY: lds_copy(L, xl, tl, tid); break;
        case OP_DR:
        case OP_PROLONG:
        case OP_OMEGA: {
          const Level<T> C = Ls[l + 1];
          MG_LDS T* xc = lds + offs[l + 1];
          if (type == OP_DR) {
            lds_dr<T, K, B1>(L, xl, bl, bands, C, xc, xc + C.nx * C.ny, tid);
          } else if (type == OP_PROLONG) {
            lds_prolong(L, xl, C, xc, tid, arg != 0, wsh[l]);
          } else {
            double s1 = 0.0, s2 = 0.0;
            lds_energy<T, K, B1>(L, xl, bl, bands, C, xc, tid, s1, s2);
            s1 = block_sum(s1, esh);
            s2 = block_sum(s2, esh);
            if (tid == 0) wsh[l] = (T)(s2 != 0.0 ? s1 / s2 : 1.0);
          }
          break;
        }
        case OP_COARSE:
          if (ncu <= COARSE_LDS_MAX)
            lds_coarse(L, xl, bl, lds_cast<double>(ainv_sh), ncu, tid);
          else
            body_coarse(L, chol[slot], ncu, tid, SUB_NT);
          break;
        case OP_LINE: lds_line<T, K, B1>(L, xl, bl, tl, bands, lds + soff, arg, omega, tid); break;
        default: break;
      }
    } else {
      switch (type) {
        case OP_COLOR: body_colour<T, false>(L, arg, ncol, omega, tid, SUB_NT); break;
        case OP_SMOOTH: {
          const int nsw = arg & SM_NSW;
          if (arg & SM_PRO) {
            body_prolong(L, Ls[l + 1], tid, SUB_NT, (arg & SM_WTD) != 0, wsh[l]);
            __syncthreads();
          }
          for (int k2 = 0; k2 < nsw * ncol; ++k2) {
            body_colour<T, false>(L, k2 % ncol, ncol, omega, tid, SUB_NT);
            if (k2 + 1 < nsw * ncol) __syncthreads();
          }
          if (arg & SM_DR) {
            __syncthreads();
            body_dr<T, false>(L, Ls[l + 1], tid, SUB_NT);
          }
          break;
        }
        case OP_JACOBI: body_jacobi<T, false>(L, arg, omega, tid, SUB_NT); break;
        case OP_COPY: body_copy(L, tid, SUB_NT); break;
        case OP_DR: body_dr<T, false>(L, Ls[l + 1], tid, SUB_NT); break;
        case OP_PROLONG: body_prolong(L, Ls[l + 1], tid, SUB_NT, arg != 0, wsh[l]); break;
        case OP_OMEGA: {
          double s1 = 0.0, s2 = 0.0;
          body_energy<KDYN, false>(L, L.x, Ls[l + 1], tid, SUB_NT, s1, s2);
          s1 = block_sum(s1, esh);
          s2 = block_sum(s2, esh);
          if (tid == 0) wsh[l] = (T)(s2 != 0.0 ? s1 / s2 : 1.0);
          break;
        }
        case OP_COARSE: body_coarse(L, chol[slot], ncu, tid, SUB_NT); break;
        case OP_LINE:
          for (int t0 = 0; t0 < L.nx + L.ny; t0 += SUB_NT) line_thomas<T, K, false>(L, arg, omega, t0 + tid);
          break;
        default: break;
      }
    }
    __syncthreads();
  }
  if (IN_LDS) {
    const Level<T> G = Ls[top];
    const int lo = row_lo(G), nr = row_hi(G) - lo + 1, ni = G.nx - 2, n = nr * ni;
    const MG_LDS T* xl = lds + offs[top];
    for (int idx = tid; idx < n; idx += SUB_NT) {
      const int r = idx / ni;
      const int i = idx - r * ni + 1, j = lo + r;
      G.x[(size_t)j * G.pitch + i] = xl[j * G.nx + i];
    }
  }
}

// --------------------------------------------------------------------------- residual norm

// Workgroup sum of v (fixed tree order); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
  }
  __syncthreads();
  return s;
}

// Stopping test from the partial sums of a norm reduction (one workgroup per
// problem slot, launched after the kernel that wrote the partials).  Thread
// t sums partials t, t + NT, ... in order, then a fixed tree: the result does
// not depend on scheduling.
template <typename T>
__global__ void __launch_bounds__(NT) k_norm_finish(const Level<T>* __restrict__ Ls, int nblocks, int mode) {
  __shared__ double sh[NT / 64];
  SolveState* st = Ls[blockIdx.z].st;
  if ((mode == NORM_CHECK || mode == NORM_LAG) && st->done) return;
  if (mode == NORM_LAG && !st->pending) return;  // this iterate's test was taken
  double v = 0.0;
  for (int k = threadIdx.x; k < nblocks; k += NT) v += st->partial[k];
  const double s = block_sum(v, sh);
  if (threadIdx.x != 0) return;
  const double nrm = sqrt(s);
  st->prev = st->last;
  st->last = nrm;
  if (mode == NORM_INIT) {
    st->r0 = nrm;
    st->cycles = 0;
    st->pending = 0;
    if (st->hist_cap > 0) st->history[0] = nrm;
    st->done = (nrm == 0.0) ? 1 : 0;
  } else if (mode == NORM_CHECK || mode == NORM_LAG) {
    st->pending = 0;
    const int c = st->cycles + 1;
    st->cycles = c;
    if (c < st->hist_cap) st->history[c] = nrm;
    if (nrm <= st->tol * st->r0)
      st->done = 1;
    else if (!(nrm <= DIVERGENCE_FACTOR * st->r0))  // also catches NaN
      st->done = 2;
  }
}

// r = b - A x on level L (FP64 accumulation), boundary x read as 0.
// Optional outputs: r (pitch L.pitch) and, for the mixed-precision outer
// step, (float) r into the FP32 finest level's b of the same slot (R32s).
// Writes one partial sum of squares per workgroup; k_norm_finish completes
// the norm.
template <typename T, int K, bool B1>
__global__ void __launch_bounds__(NT) k_resnorm(const Level<T>* __restrict__ Ls, int mode, T* __restrict__ rout,
                                                const Level<float>* __restrict__ R32s, int nbx, int rows_per_block) {
  constexpr int RB = 4;  // rows whose loads a thread issues together
  __shared__ double sh[NT / 64];
  const Level<T> L = Ls[blockIdx.z];
  SolveState* st = L.st;
  if (mode == NORM_CHECK && st->done) return;
  float* r32 = R32s ? R32s[blockIdx.z].b : nullptr;
  const int p32 = R32s ? R32s[blockIdx.z].pitch : 0;
  const int lo = row_lo(L), hi = row_hi(L), ni = L.nx - 2;
  // block = (column chunk, row group); thread = one column, marching up the
  // group's rows with a 3x3 window of x in registers.  A Dirichlet boundary
  // node reads as 0 whatever the caller stored there.
  const int bx = blockIdx.x % nbx, by = blockIdx.x / nbx;
  const int i = 1 + bx * NT + threadIdx.x;
  const bool act = i <= ni;
  const int ic = act ? i : 1;  // in-range column for lanes past the row end (their results are dropped)
  const bool wok = ic > 1, eok = ic < ni;
  const int j0 = lo + by * rows_per_block, j1 = min(hi, j0 + rows_per_block - 1);
  Cf<T> col{};
  if (K == ST9 && B1) col = coefs<K>(L, ic, 0, 0);
  auto load_row = [&](int r, T* w) {  // x at columns ic-1, ic, ic+1 of stored row r (wrapped)
    const bool bnd = !L.py && (r == 0 || r == L.ny - 1);
    const T* xr = L.x + (size_t)r * L.pitch;
    w[0] = (!bnd && wok) ? xr[ic - 1] : (T)0;
    w[1] = !bnd ? xr[ic] : (T)0;
    w[2] = (!bnd && eok) ? xr[ic + 1] : (T)0;
  };
  double acc = 0.0;
  if (j0 <= j1) {
    T ws[3], wc[3];
    load_row(wrap_dn(j0, L.ny, L.py), ws);
    load_row(j0, wc);
    for (int j = j0; j <= j1; j += RB) {
      T wn[RB][3], bp[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int jj = j + u;
        if (jj > j1) break;
        load_row(wrap_up(jj, L.ny, L.py), wn[u]);
        bp[u] = L.b[(size_t)jj * L.pitch + ic];
      }
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int jj = j + u;
        if (jj > j1) break;
        Nbr<T> v;
        v.sw = ws[0];
        v.s = ws[1];
        v.se = ws[2];
        v.w = wc[0];
        v.c = wc[1];
        v.e = wc[2];
        v.nw = wn[u][0];
        v.n = wn[u][1];
        v.ne = wn[u][2];
        const Cf<T> a = (K == ST9 && !B1) ? coefs<K>(L, ic, jj, wrap_dn(jj, L.ny, L.py)) : col;
        const T d = defect_v<K>(L, a, v, bp[u]);
        if (act) {
          if (rout) rout[(size_t)jj * L.pitch + i] = d;
          if (r32) r32[(size_t)jj * p32 + i] = (float)d;
          acc += (double)d * (double)d;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          ws[c] = wc[c];
          wc[c] = wn[u][c];
        }
      }
    }
  }
  const double part = block_sum(acc, sh);
  if (threadIdx.x == 0) st->partial[blockIdx.x] = part;
}

// Mixed precision outer update: x (FP64) += e (FP32), e = 0.
__global__ void __launch_bounds__(NT) k_outer_update(const Level<double>* __restrict__ L64s,
                                                     const Level<float>* __restrict__ L32s) {
  const Level<double> X = L64s[blockIdx.z];
  if (X.st->done) return;
  const Level<float> E = L32s[blockIdx.z];
  const int lo = row_lo(X), nr = row_hi(X) - lo + 1, ni = X.nx - 2;
  const int n = nr * ni;
  for (int idx = blockIdx.x * NT + threadIdx.x; idx < n; idx += gridDim.x * NT) {
    const int r = idx / ni;
    const int i = idx - r * ni + 1;
    const int j = lo + r;
    float* ep = E.x + (size_t)j * E.pitch + i;
    X.x[(size_t)j * X.pitch + i] += (double)(*ep);
    *ep = 0.0f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) X.st->pending = 1;
}

// Zero the Dirichlet boundary nodes of x.
__global__ void k_zero_boundary(double* x, int nx, int ny, int pitch, int py) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ny) {
    x[(size_t)t * pitch] = 0.0;
    x[(size_t)t * pitch + nx - 1] = 0.0;
  }
  if (!py && t < nx) {
    x[t] = 0.0;
    x[(size_t)(ny - 1) * pitch + t] = 0.0;
  }
}

// --------------------------------------------------------------------------- setup kernels

// Cell coefficients of a refined tensor grid folded into the equidistant
// form: cell (i, j) of size hx_c = rx[i] hx0 by hy_c = ry[j] hy0 contributes
// kx hy_c/hx_c K1 (x) M1 + ky hx_c/hy_c M1 (x) K1 over hx0 hy0, which is the
// equidistant cell's kx'/hx0^2 K1 (x) M1 + ky'/hy0^2 M1 (x) K1 with kx' = kx
// ry/rx and ky' = ky rx/ry.  Input [ncy][ncx] (or [ncx] when in_oned), output
// nrows rows of ncx.
__global__ void k_graded_cells(const double* __restrict__ kx, const double* __restrict__ ky, int in_oned,
                               const double* __restrict__ rx, const double* __restrict__ ry, double* __restrict__ kxo,
                               double* __restrict__ kyo, int ncx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= ncx) return;
  const size_t src = in_oned ? (size_t)i : (size_t)j * ncx + i, dst = (size_t)j * ncx + i;
  const double q = ry[j] / rx[i];
  kxo[dst] = kx[src] * q;
  kyo[dst] = ky[src] / q;
}


// Q1 bands C, E, N, NE, NW at every stored node from per-cell kx, ky
// (cell (ci, cj) at kx[cj * kpitch + ci]; kpitch = 0 when they vary along x
// only, then only row 0 of the bands is written).  Element matrix of a cell,
// divided by hx*hy: kx/hx^2 K1 (x) M1 + ky/hy^2 M1 (x) K1 with K1 = [1 -1; -1 1],
// M1 = [1/3 1/6; 1/6 1/3].
__global__ void k_q1_bands(double* band, int bstride, int bpitch, int nrows, int nx, int ny, int py,
                           const double* __restrict__ kx, const double* __restrict__ ky, int kpitch, double hx,
                           double hy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= nx || j >= nrows) return;
  const int ncx = nx - 1, ncy = py ? ny : ny - 1;
  const double ax = 1.0 / (hx * hx), ay = 1.0 / (hy * hy);
  // cells around node (i, j): SW (i-1, j-1), SE (i, j-1), NW (i-1, j), NE (i, j)
  auto cell = [&](int ci, int cj, double& cx, double& cy) -> bool {
    if (ci < 0 || ci >= ncx) return false;
    if (py) {
      cj = (cj + ncy) % ncy;
    } else if (cj < 0 || cj >= ncy) {
      return false;
    }
    const size_t c = (size_t)cj * kpitch + ci;
    cx = kx[c] * ax;
    cy = ky[c] * ay;
    return true;
  };
  // with kpitch == 0 every row sees the same cells; evaluate at an interior row
  const int jj = (kpitch == 0 && !py) ? 1 : j;
  double C = 0, E = 0, N = 0, NE = 0, NW = 0, cx, cy;
  if (cell(i - 1, jj - 1, cx, cy)) C += (cx + cy) / 3.0;
  if (cell(i, jj - 1, cx, cy)) { C += (cx + cy) / 3.0; E += -cx / 3.0 + cy / 6.0; }
  if (cell(i - 1, jj, cx, cy)) { C += (cx + cy) / 3.0; N += cx / 6.0 - cy / 3.0; NW += -(cx + cy) / 6.0; }
  if (cell(i, jj, cx, cy)) {
    C += (cx + cy) / 3.0;
    E += -cx / 3.0 + cy / 6.0;
    N += cx / 6.0 - cy / 3.0;
    NE += -(cx + cy) / 6.0;
  }
  const size_t p = (size_t)j * bpitch + i;
  band[p] = C;
  band[bstride + p] = E;
  band[2 * (size_t)bstride + p] = N;
  band[3 * (size_t)bstride + p] = NE;
  band[4 * (size_t)bstride + p] = NW;
}

// Fine coefficient a_pq for q = p + (s, t) from the symmetric band storage.
__device__ double band_coef(const double* band, int bstride, int bpitch, int nx, int ny, int py, int i, int j, int s,
                            int t) {
  auto idx = [&](int ii, int jj) -> size_t {
    if (py) jj = (jj % ny + ny) % ny;
    return (size_t)(bpitch ? jj : 0) * bpitch + ii;
  };
  const double* C = band;
  const double* E = band + bstride;
  const double* N = band + 2 * (size_t)bstride;
  const double* NE = band + 3 * (size_t)bstride;
  const double* NW = band + 4 * (size_t)bstride;
  if (s == 0 && t == 0) return C[idx(i, j)];
  if (s == 1 && t == 0) return E[idx(i, j)];
  if (s == -1 && t == 0) return E[idx(i - 1, j)];
  if (s == 0 && t == 1) return N[idx(i, j)];
  if (s == 0 && t == -1) return N[idx(i, j - 1)];
  if (s == 1 && t == 1) return NE[idx(i, j)];
  if (s == -1 && t == -1) return NE[idx(i - 1, j - 1)];
  if (s == -1 && t == 1) return NW[idx(i, j)];
  return NW[idx(i + 1, j - 1)];  // s == 1, t == -1
}

// Galerkin coarse bands A_H = R A_h P at coarse node (I, J): for each of the
// couplings C, E, N, NE, NW to c' = (I, J) + (dI, dJ),
//   sum_{p in supp R(I,J)} w_p sum_{q ~ p} a_pq P(q, c'),
// with full-weighting weights w and bilinear weights P.  Couplings to a
// Dirichlet boundary node are stored as 0.
__global__ void k_rap(double* cband, int cbstride, int cbpitch, int cnrows, int ncx_nodes, int ncy_nodes,
                      const double* __restrict__ fband, int fbstride, int fbpitch, int nxf, int nyf, int py) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y;
  if (I >= ncx_nodes || J >= cnrows) return;
  const int offs[5][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}, {-1, 1}};
  const double w[3] = {0.25, 0.5, 0.25};
  // rows of a 1-D band are evaluated at an interior row
  const int JJ = (cbpitch == 0 && !py) ? 1 : J;
  const bool interior_I = I >= 1 && I <= ncx_nodes - 2;
  const bool interior_J = py || (JJ >= 1 && JJ <= ncy_nodes - 2);
  for (int k = 0; k < 5; ++k) {
    const int Ic = I + offs[k][0];
    int Jc = JJ + offs[k][1];
    double v = 0.0;
    const bool tgt_in = Ic >= 1 && Ic <= ncx_nodes - 2 && (py || (Jc >= 1 && Jc <= ncy_nodes - 2));
    if (interior_I && interior_J && tgt_in) {
      for (int b = -1; b <= 1; ++b) {
        for (int a = -1; a <= 1; ++a) {
          const int pi = 2 * I + a;
          int pj = 2 * JJ + b;
          if (py) pj = (pj + nyf) % nyf;
          const double wp = w[a + 1] * w[b + 1];
          for (int t = -1; t <= 1; ++t) {
            for (int s = -1; s <= 1; ++s) {
              const int qi = pi + s;
              const int qj = pj + t;  // unwrapped; compared with 2 Jc modulo nyf below
              int dx = qi - 2 * Ic;
              int dy = qj - 2 * Jc;
              if (py) {
                dy = ((dy % nyf) + nyf) % nyf;
                if (dy > nyf / 2) dy -= nyf;
              }
              if (dx < -1 || dx > 1 || dy < -1 || dy > 1) continue;
              const double pw = (dx == 0 ? 1.0 : 0.5) * (dy == 0 ? 1.0 : 0.5);
              const double a_pq = band_coef(fband, fbstride, fbpitch, nxf, nyf, py, pi, pj, s, t);
              v += wp * a_pq * pw;
            }
          }
        }
      }
    } else if (k == 0) {
      v = 1.0;  // keep the diagonal of non-unknown nodes finite and non-zero
    }
    cband[(size_t)k * cbstride + (size_t)J * cbpitch + I] = v;
  }
}

// Dense matrix of the coarsest operator over its unknowns (row by row).
__global__ void k_dense_coarse(double* A, int n, int nx, int ny, int py, int kind, double cx, double cy, double dg,
                               const double* __restrict__ band, int bstride, int bpitch) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int ni = nx - 2, lo = py ? 0 : 1, hi = py ? ny - 1 : ny - 2;
  const int r = k / ni;
  const int i = k - r * ni + 1, j = lo + r;
  for (int t = -1; t <= 1; ++t) {
    for (int s = -1; s <= 1; ++s) {
      double a;
      if (kind == ST5) {
        if (s == 0 && t == 0) a = dg;
        else if (t == 0) a = -cx;
        else if (s == 0) a = -cy;
        else a = 0.0;
      } else {
        a = band_coef(band, bstride, bpitch, nx, ny, py, i, j, s, t);
      }
      const int qi = i + s;
      int qj = j + t;
      if (py) qj = (qj + ny) % ny;
      if (qi < 1 || qi > nx - 2 || qj < lo || qj > hi) continue;
      const int q = (qj - lo) * ni + (qi - 1);
      A[(size_t)k * n + q] += a;
    }
  }
}

// In-place Cholesky A = L L^T (lower triangle of A), one workgroup.  info[0]
// is set to k + 1 when the k-th pivot is not positive.
__global__ void k_cholesky(double* A, int n, int* info) {
  const int tid = threadIdx.x, nth = blockDim.x;
  __shared__ int bad;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      const double d = A[(size_t)k * n + k];
      if (!(d > 0.0)) {
        bad = k + 1;
      } else {
        A[(size_t)k * n + k] = sqrt(d);
      }
    }
    __syncthreads();
    if (bad) break;
    const double dk = A[(size_t)k * n + k];
    for (int r = k + 1 + tid; r < n; r += nth) A[(size_t)r * n + k] /= dk;
    __syncthreads();
    const int m = n - k - 1;
    for (int e = tid; e < m * m; e += nth) {
      const int r = k + 1 + e / m, c = k + 1 + e % m;
      if (c <= r) A[(size_t)r * n + c] -= A[(size_t)r * n + k] * A[(size_t)c * n + k];
    }
    __syncthreads();
  }
  if (tid == 0) info[0] = bad;
}

// Inverse of A = L L^T from its Cholesky factor (lower, row-major): one
// thread per column c solves L y = e_c, L^T x = y and writes x as row c of
// the (symmetric) inverse.  Setup only.
__global__ void k_chol_inverse(const double* __restrict__ Lf, double* __restrict__ X, int n) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double* x = X + (size_t)c * n;
  for (int k = 0; k < c; ++k) x[k] = 0.0;
  for (int k = c; k < n; ++k) {
    double s = k == c ? 1.0 : 0.0;
    for (int j = c; j < k; ++j) s -= Lf[(size_t)k * n + j] * x[j];
    x[k] = s / Lf[(size_t)k * n + k];
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = x[k];
    for (int j = k + 1; j < n; ++j) s -= Lf[(size_t)j * n + k] * x[j];
    x[k] = s / Lf[(size_t)k * n + k];
  }
}

// Counts entries of v that are not finite or not > 0.
__global__ void k_count_bad(const double* __restrict__ v, long n, int* count) {
  int bad = 0;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const double a = v[k];
    if (!(a > 0.0) || !(a < INFINITY)) ++bad;
  }
  if (bad) atomicAdd(count, bad);
}

// Counts non-finite entries of the unknowns of a node array.
__global__ void k_count_nonfinite(const double* __restrict__ v, int nx, int ny, int pitch, int py, int* count) {
  const int lo = py ? 0 : 1, nr = (py ? ny - 1 : ny - 2) - lo + 1, ni = nx - 2;
  const long n = (long)nr * ni;
  int bad = 0;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
    const long r = idx / ni;
    const double a = v[(size_t)(lo + r) * pitch + (idx - r * ni + 1)];
    if (!(a - a == 0.0)) ++bad;
  }
  if (bad) atomicAdd(count, bad);
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ s, D* __restrict__ d, long n) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) d[k] = (D)s[k];
}

// Inverse-diagonal band D = 1 / C (0 where C is 0: entries no unknown reads).
__global__ void k_inv_diag(const double* __restrict__ c, double* __restrict__ d, long n) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
    d[k] = c[k] != 0.0 ? 1.0 / c[k] : 0.0;
}

// dL/dk for each cell: -lam_e^T K u_e with K = Ex + Ey the unit-coefficient
// element matrix (local node order 2 b + a, a along x).
__global__ void k_coeff_grad(const double* __restrict__ u, const double* __restrict__ lam, double* __restrict__ g,
                             int nx, int ny, int py, double hx, double hy) {
  const int ci = blockIdx.x * blockDim.x + threadIdx.x;
  const int cj = blockIdx.y;
  const int ncx = nx - 1, ncy = py ? ny : ny - 1;
  if (ci >= ncx || cj >= ncy) return;
  const int j0 = cj, j1 = (py && cj + 1 == ny) ? 0 : cj + 1;
  const double ue[4] = {u[(size_t)j0 * nx + ci], u[(size_t)j0 * nx + ci + 1], u[(size_t)j1 * nx + ci],
                        u[(size_t)j1 * nx + ci + 1]};
  const double le[4] = {lam[(size_t)j0 * nx + ci], lam[(size_t)j0 * nx + ci + 1], lam[(size_t)j1 * nx + ci],
                        lam[(size_t)j1 * nx + ci + 1]};
  const double K1[2][2] = {{1.0, -1.0}, {-1.0, 1.0}};
  const double M1[2][2] = {{1.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 1.0 / 3.0}};
  const double ax = 1.0 / (hx * hx), ay = 1.0 / (hy * hy);
  double s = 0.0;
  for (int p = 0; p < 4; ++p) {
    const int a = p & 1, b = p >> 1;
    double kp = 0.0;
    for (int q = 0; q < 4; ++q) {
      const int a2 = q & 1, b2 = q >> 1;
      kp += (ax * K1[a][a2] * M1[b][b2] + ay * M1[a][a2] * K1[b][b2]) * ue[q];
    }
    s += le[p] * kp;
  }
  g[(size_t)cj * ncx + ci] = -s;
}

// --------------------------------------------------------------------------- launchers

static inline unsigned blocks_for(long n, int per = NT) { return (unsigned)((n + per - 1) / per); }

template <typename T>
hipError_t launch_colour(const Level<T>* Ls, const LevelShape& s, int c, int ncol, T omega, int nslots,
                         hipStream_t st) {
  const int nk = (s.nx - 1) / 2 + 1;
  const int nrows = ncol == 2 ? s.nrows : (s.nrows + 1) / 2;
  hipLaunchKernelGGL(k_colour<T>, dim3(blocks_for((long)nk * nrows), 1, nslots), dim3(NT), 0, st, Ls, c, ncol, omega);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_jacobi(const Level<T>* Ls, const LevelShape& s, int dir, T omega, int nslots, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi<T>, dim3(blocks_for((long)(s.nx - 2) * s.nrows), 1, nslots), dim3(NT), 0, st, Ls, dir,
                     omega);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const Level<T>* Ls, const LevelShape& s, int nslots, hipStream_t st) {
  hipLaunchKernelGGL(k_copy<T>, dim3(blocks_for((long)(s.nx - 2) * s.nrows), 1, nslots), dim3(NT), 0, st, Ls);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dr(const Level<T>* Fs, const Level<T>* Cs, const LevelShape& c, int nslots, hipStream_t st) {
  hipLaunchKernelGGL(k_dr<T>, dim3(blocks_for((long)(c.nx - 2) * c.nrows), 1, nslots), dim3(NT), 0, st, Fs, Cs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_energy(const Level<T>* Fs, const Level<T>* Cs, const LevelShape& f, int src_t, int kind, int nslots,
                         hipStream_t st) {
  int nb = blocks_for((long)(f.nx - 2) * f.nrows);
  if (nb > MAX_NORM_BLOCKS / 2) nb = MAX_NORM_BLOCKS / 2;  // two partial sums per workgroup
  auto k = kind == ST5 ? k_energy<T, ST5> : k_energy<T, ST9>;
  hipLaunchKernelGGL(k, dim3(nb, 1, nslots), dim3(NT), 0, st, Fs, Cs, src_t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_finish<T>, dim3(1, 1, nslots), dim3(NT), 0, st, Fs, nb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const Level<T>* Fs, const Level<T>* Cs, const LevelShape& f, int weighted, int nslots,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_prolong<T>, dim3(blocks_for((long)(f.nx - 2) * f.nrows), 1, nslots), dim3(NT), 0, st, Fs, Cs,
                     weighted);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse(const Level<T>* Ls, const double* const* chol, int n, int nslots, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse<T>, dim3(1, 1, nslots), dim3(NT), 0, st, Ls, chol, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_subcycle(const Level<T>* levs, int nlev, const DOp* prog, const int* beg, const int* cnt,
                           const double* const* chol, int ncu, T omega, int ncol, int nslots, hipStream_t st) {
  hipLaunchKernelGGL((k_subcycle<T, false, KDYN>), dim3(1, 1, nslots), dim3(SUB_NT), 0, st, levs, nlev, 0, prog, beg,
                     cnt, chol, ncu, omega, ncol, 0);
  return hipGetLastError();
}

template <typename T>
hipError_t prepare_subcycle_lds() {
  const void* ks[3] = {(const void*)k_subcycle<T, true, ST5>, (const void*)k_subcycle<T, true, ST9>,
                       (const void*)k_subcycle<T, true, ST9, true>};
  for (const void* k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)SUB_LDS_BUDGET);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_subcycle_lds(const Level<T>* levs, int nlev, int top, const DOp* prog, const int* beg,
                               const int* cnt, const double* const* chol, int ncu, T omega, int ncol, int narr,
                               int kind, bool oned, size_t lds_bytes, int nslots, hipStream_t st) {
  auto k = kind == ST5 ? k_subcycle<T, true, ST5>
                       : (oned ? k_subcycle<T, true, ST9, true> : k_subcycle<T, true, ST9, false>);
  hipLaunchKernelGGL(k, dim3(1, 1, nslots), dim3(SUB_NT), lds_bytes, st, levs, nlev, top, prog, beg, cnt, chol, ncu,
                     omega, ncol, narr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_norm_finish(const Level<T>* Ls, int nblocks, int mode, int nslots, hipStream_t st) {
  hipLaunchKernelGGL(k_norm_finish<T>, dim3(1, 1, nslots), dim3(NT), 0, st, Ls, nblocks, mode);
  return hipGetLastError();
}

int norm_blocks(const LevelShape& s) {
  const long n = (long)(s.nx - 2) * s.nrows;
  long b = (n + NT * 4 - 1) / (NT * 4);
  if (b < 1) b = 1;
  if (b > MAX_NORM_BLOCKS) b = MAX_NORM_BLOCKS;
  return (int)b;
}

template <typename T>
hipError_t launch_resnorm(const Level<T>* Ls, const LevelShape& s, int mode, T* rout, const Level<float>* R32s,
                          int kind, bool oned, int nslots, hipStream_t st) {
  const int nbx = (s.nx - 2 + NT - 1) / NT;
  const int maxby = MAX_NORM_BLOCKS / nbx > 0 ? MAX_NORM_BLOCKS / nbx : 1;
  const int rpb = (s.nrows + maxby - 1) / maxby;
  const int nb = nbx * ((s.nrows + rpb - 1) / rpb);
  if (nb > MAX_NORM_BLOCKS) return hipErrorInvalidValue;
  auto k = kind == ST5 ? k_resnorm<T, ST5, false> : (oned ? k_resnorm<T, ST9, true> : k_resnorm<T, ST9, false>);
  hipLaunchKernelGGL(k, dim3(nb, 1, nslots), dim3(NT), 0, st, Ls, mode, rout, R32s, nbx, rpb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_norm_finish<T>(Ls, nb, mode, nslots, st);
}

hipError_t launch_outer_update(const Level<double>* L64, const Level<float>* L32, const LevelShape& s, int nslots,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_outer_update, dim3(blocks_for((long)(s.nx - 2) * s.nrows), 1, nslots), dim3(NT), 0, st, L64,
                     L32);
  return hipGetLastError();
}

hipError_t launch_zero_boundary(double* x, int nx, int ny, int pitch, int py, hipStream_t st) {
  const int n = nx > ny ? nx : ny;
  hipLaunchKernelGGL(k_zero_boundary, dim3(blocks_for(n)), dim3(NT), 0, st, x, nx, ny, pitch, py);
  return hipGetLastError();
}

hipError_t launch_graded_cells(const double* kx, const double* ky, int in_oned, const double* rx, const double* ry,
                               double* kxo, double* kyo, int ncx, int nrows, hipStream_t st) {
  hipLaunchKernelGGL(k_graded_cells, dim3(blocks_for(ncx), nrows), dim3(NT), 0, st, kx, ky, in_oned, rx, ry, kxo, kyo,
                     ncx);
  return hipGetLastError();
}

hipError_t launch_q1_bands(double* band, int bstride, int bpitch, int nrows, int nx, int ny, int py, const double* kx,
                           const double* ky, int kpitch, double hx, double hy, hipStream_t st) {
  hipLaunchKernelGGL(k_q1_bands, dim3(blocks_for(nx), nrows), dim3(NT), 0, st, band, bstride, bpitch, nrows, nx, ny, py,
                     kx, ky, kpitch, hx, hy);
  return hipGetLastError();
}

hipError_t launch_rap(double* cband, int cbstride, int cbpitch, int cnrows, int ncx, int ncy, const double* fband,
                      int fbstride, int fbpitch, int nxf, int nyf, int py, hipStream_t st) {
  hipLaunchKernelGGL(k_rap, dim3(blocks_for(ncx), cnrows), dim3(NT), 0, st, cband, cbstride, cbpitch, cnrows, ncx, ncy,
                     fband, fbstride, fbpitch, nxf, nyf, py);
  return hipGetLastError();
}

hipError_t launch_dense_coarse(double* A, int n, int nx, int ny, int py, int kind, double cx, double cy, double dg,
                               const double* band, int bstride, int bpitch, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_coarse, dim3(blocks_for(n)), dim3(NT), 0, st, A, n, nx, ny, py, kind, cx, cy, dg, band,
                     bstride, bpitch);
  return hipGetLastError();
}

hipError_t launch_cholesky(double* A, int n, int* info, hipStream_t st) {
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, st, A, n, info);
  return hipGetLastError();
}

hipError_t launch_chol_inverse(const double* Lf, double* X, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_chol_inverse, dim3((n + 63) / 64), dim3(64), 0, st, Lf, X, n);
  return hipGetLastError();
}

hipError_t launch_count_bad(const double* v, long n, int* count, hipStream_t st) {
  long b = (n + NT - 1) / NT;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_count_bad, dim3((unsigned)b), dim3(NT), 0, st, v, n, count);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const double* v, int nx, int ny, int pitch, int py, int* count, hipStream_t st) {
  long n = (long)nx * ny;
  long b = (n + NT - 1) / NT;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)b), dim3(NT), 0, st, v, nx, ny, pitch, py, count);
  return hipGetLastError();
}

hipError_t launch_to_float(const double* s, float* d, long n, hipStream_t st) {
  long b = (n + NT - 1) / NT;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)b), dim3(NT), 0, st, s, d, n);
  return hipGetLastError();
}

hipError_t launch_inv_diag(double* band, int bstride, hipStream_t st) {
  long b = (bstride + NT - 1) / NT;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_inv_diag, dim3((unsigned)b), dim3(NT), 0, st, band, band + (size_t)BAND_D * bstride,
                     (long)bstride);
  return hipGetLastError();
}

hipError_t launch_coeff_grad(const double* u, const double* lam, double* g, int nx, int ny, int py, double hx,
                             double hy, hipStream_t st) {
  const int ncy = py ? ny : ny - 1;
  hipLaunchKernelGGL(k_coeff_grad, dim3(blocks_for(nx - 1), ncy), dim3(NT), 0, st, u, lam, g, nx, ny, py, hx, hy);
  return hipGetLastError();
}

#define MG_INSTANTIATE(T)                                                                                          \
  template hipError_t launch_colour<T>(const Level<T>*, const LevelShape&, int, int, T, int, hipStream_t);           \
  template hipError_t launch_jacobi<T>(const Level<T>*, const LevelShape&, int, T, int, hipStream_t);             \
  template hipError_t launch_copy<T>(const Level<T>*, const LevelShape&, int, hipStream_t);                       \
  template hipError_t launch_dr<T>(const Level<T>*, const Level<T>*, const LevelShape&, int, hipStream_t);        \
  template hipError_t launch_prolong<T>(const Level<T>*, const Level<T>*, const LevelShape&, int, int, hipStream_t); \
  template hipError_t launch_energy<T>(const Level<T>*, const Level<T>*, const LevelShape&, int, int, int,       \
                                       hipStream_t);                                                            \
  template hipError_t launch_coarse<T>(const Level<T>*, const double* const*, int, int, hipStream_t);             \
  template hipError_t launch_line_factor<T>(const Level<T>&, int, hipStream_t);                                    \
  template hipError_t prepare_line_cr<T>();                                                                        \
  template hipError_t launch_line<T>(const Level<T>*, const LevelShape&, int, T, int, int, hipStream_t);          \
  template hipError_t launch_subcycle<T>(const Level<T>*, int, const DOp*, const int*, const int*,                \
                                         const double* const*, int, T, int, int, hipStream_t);                     \
  template hipError_t launch_resnorm<T>(const Level<T>*, const LevelShape&, int, T*, const Level<float>*, int, bool, \
                                        int, hipStream_t);                                                          \
  template hipError_t prepare_subcycle_lds<T>();                                                                   \
  template hipError_t launch_norm_finish<T>(const Level<T>*, int, int, int, hipStream_t);                          \
  template hipError_t launch_subcycle_lds<T>(const Level<T>*, int, int, const DOp*, const int*, const int*,        \
                                             const double* const*, int, T, int, int, int, bool, size_t, int,      \
                                             hipStream_t);

MG_INSTANTIATE(double)
MG_INSTANTIATE(float)

}  // namespace mg
