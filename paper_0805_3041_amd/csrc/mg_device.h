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
  const T* band;          // ST9: bands C, E, N, NE, NW, each `bstride` apart
  int bpitch;             // ST9: band row pitch (0: one row for every j)
  int bstride;
  SolveState* st;         // owning problem's state
};

// Host-built op of the coarse-level interpreter (one workgroup runs a list).
enum OpType {
  OP_COLOR = 0,     // Gauss-Seidel update of colour `arg` on `level`
  OP_JACOBI = 1,    // damped Jacobi x -> t (arg = 0) or t -> x (arg = 1)
  OP_COPY = 2,      // x <- t on `level`
  OP_DR = 3,        // restrict the defect of `level` into b of level+1, zero x of level+1
  OP_PROLONG = 4,   // x(level) += P x(level+1)
  OP_COARSE = 5,    // exact solve on the coarsest `level`
};

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

// Value of x at stored node (i, j); with MASK a Dirichlet boundary node reads
// as 0 whatever is stored there (used where x comes from the caller).
template <bool MASK, typename T>
__device__ __forceinline__ T xval(const Level<T>& L, const T* __restrict__ x, int i, int j) {
  if (MASK && (i == 0 || i == L.nx - 1 || (!L.py && (j == 0 || j == L.ny - 1)))) return (T)0;
  return x[(size_t)j * L.pitch + i];
}

// Sum over the neighbours q != p of a_pq x_q at interior node (i, j) of level L.
// Rows jm, jp are j's wrapped neighbours.
template <bool MASK = false, typename T>
__device__ __forceinline__ T offdiag_sum(const Level<T>& L, const T* __restrict__ x, int i, int j, int jm, int jp) {
  if (L.kind == ST5) {
    const T xw = xval<MASK>(L, x, i - 1, j), xe = xval<MASK>(L, x, i + 1, j);
    const T xs = xval<MASK>(L, x, i, jm), xn = xval<MASK>(L, x, i, jp);
    return -(L.cx * (xw + xe) + L.cy * (xs + xn));
  }
  const int BP = L.bpitch;
  const T* E = bandp(L, 1);
  const T* N = bandp(L, 2);
  const T* NE = bandp(L, 3);
  const T* NW = bandp(L, 4);
  const size_t rp = (size_t)j * BP, rs = (size_t)jm * BP;
  T s = E[rp + i] * xval<MASK>(L, x, i + 1, j) + E[rp + i - 1] * xval<MASK>(L, x, i - 1, j);
  s += N[rp + i] * xval<MASK>(L, x, i, jp) + N[rs + i] * xval<MASK>(L, x, i, jm);
  s += NE[rp + i] * xval<MASK>(L, x, i + 1, jp) + NE[rs + i - 1] * xval<MASK>(L, x, i - 1, jm);
  s += NW[rp + i] * xval<MASK>(L, x, i - 1, jp) + NW[rs + i + 1] * xval<MASK>(L, x, i + 1, jm);
  return s;
}

template <typename T>
__device__ __forceinline__ T diag_at(const Level<T>& L, int i, int j) {
  if (L.kind == ST5) return L.dg;
  return bandp(L, 0)[(size_t)j * L.bpitch + i];
}

// Gauss-Seidel value of node (i, j): (b_p - sum_{q != p} a_pq x_q) / a_pp.
template <typename T>
__device__ __forceinline__ T gs_value(const Level<T>& L, const T* __restrict__ x, const T* __restrict__ b,
                                      int i, int j, int jm, int jp) {
  const T off = offdiag_sum(L, x, i, j, jm, jp);
  const T rhs = b[(size_t)j * L.pitch + i] - off;
  if (L.kind == ST5) return rhs * L.inv_dg;
  return rhs / diag_at(L, i, j);
}

// Defect b_p - (A x)_p at interior node (i, j).
template <bool MASK = false, typename T>
__device__ __forceinline__ T defect_at(const Level<T>& L, const T* __restrict__ x, const T* __restrict__ b,
                                       int i, int j, int jm, int jp) {
  const size_t p = (size_t)j * L.pitch + i;
  return b[p] - (diag_at(L, i, j) * x[p] + offdiag_sum<MASK>(L, x, i, j, jm, jp));
}

// Damped Jacobi value: x_p + omega (b - A x)_p / a_pp.
template <typename T>
__device__ __forceinline__ T jacobi_value(const Level<T>& L, const T* __restrict__ x, const T* __restrict__ b,
                                          int i, int j, int jm, int jp, T omega) {
  const T d = defect_at(L, x, b, i, j, jm, jp);
  const size_t p = (size_t)j * L.pitch + i;
  if (L.kind == ST5) return x[p] + omega * d * L.inv_dg;
  return x[p] + omega * d / diag_at(L, i, j);
}

// Full-weighting restriction of the fine defect at coarse node (I, J):
// (1/16) [1 2 1; 2 4 2; 1 2 1] centred on fine node (2I, 2J).
template <typename T>
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
    const T dw = defect_at(F, x, b, i0 - 1, j, jjm, jjp);
    const T dc = defect_at(F, x, b, i0, j, jjm, jjp);
    const T de = defect_at(F, x, b, i0 + 1, j, jjm, jjp);
    acc[r] = (T)0.25 * (dw + de) + (T)0.5 * dc;
  }
  return (T)0.25 * (acc[0] + acc[2]) + (T)0.5 * acc[1];
}

// Bilinear interpolation of the coarse correction at fine node (i, j).
template <typename T>
__device__ __forceinline__ T prolong_value(const T* __restrict__ xc, int pitchc, int nyc, int py, int i, int j) {
  const int I = i >> 1, J = j >> 1;
  const bool ox = i & 1, oy = j & 1;
  const int J1 = (oy && py && J + 1 == nyc) ? 0 : J + 1;
  const T* r0 = xc + (size_t)J * pitchc;
  if (!oy) {
    if (!ox) return r0[I];
    return (T)0.5 * (r0[I] + r0[I + 1]);
  }
  const T* r1 = xc + (size_t)J1 * pitchc;
  if (!ox) return (T)0.5 * (r0[I] + r1[I]);
  return (T)0.25 * ((r0[I] + r0[I + 1]) + (r1[I] + r1[I + 1]));
}

}  // namespace mg
