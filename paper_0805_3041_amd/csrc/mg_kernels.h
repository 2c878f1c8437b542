// Host-visible launchers of the multigrid kernels (mg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "mg_device.h"

namespace mg {

constexpr int MAX_COARSE_UNKNOWNS = 1024;  // coarsest grid solved by a dense Cholesky factor
constexpr int SUB_NT = 1024;               // threads of the single-workgroup coarse-level kernel
constexpr int MAX_NORM_BLOCKS = 1024;      // workgroups of a residual-norm reduction
constexpr double DIVERGENCE_FACTOR = 1.0e6;
constexpr int MAX_LEVELS = 24;
constexpr int MAX_SUB_OPS = 1024;  // ops of a coarse-level program kept in LDS
constexpr size_t SUB_LDS_BUDGET = 140 * 1024;  // dynamic LDS of the coarse-level kernel (160 KB per CU)

// NORM_LAG: the stopping test of the iterate the norm was just formed from,
// taken only if a cycle has changed that iterate since the last test
// (SolveState::pending); the norm of a cycle's result is then formed at the
// start of the next cycle or by a check of its own.
enum NormMode { NORM_INIT = 0, NORM_CHECK = 1, NORM_RESID = 2, NORM_LAG = 3 };

// Stored shape of a level plus its number of rows that carry unknowns.
struct LevelShape {
  int nx, ny, py, nrows;
};

template <typename T>
hipError_t launch_colour(const Level<T>* Ls, const LevelShape& s, int c, int ncol, T omega, int nslots,
                         hipStream_t st);
template <typename T>
hipError_t launch_jacobi(const Level<T>* Ls, const LevelShape& s, int dir, T omega, int nslots, hipStream_t st);
template <typename T>
hipError_t launch_copy(const Level<T>* Ls, const LevelShape& s, int nslots, hipStream_t st);
template <typename T>
hipError_t launch_dr(const Level<T>* Fs, const Level<T>* Cs, const LevelShape& c, int nslots, hipStream_t st);
// x += P e on level f; weighted: x += omega_l P e with the level's adaptive weight
template <typename T>
hipError_t launch_prolong(const Level<T>* Fs, const Level<T>* Cs, const LevelShape& f, int weighted, int nslots,
                          hipStream_t st);
// adaptive omega_l of level f (written to each slot's Level::wl): the
// energy-minimising weight of the prolonged correction; x read from the
// level's t (src_t, after a fused pre-pass) or x
template <typename T>
hipError_t launch_energy(const Level<T>* Fs, const Level<T>* Cs, const LevelShape& f, int src_t, int kind, int nslots,
                         hipStream_t st);
template <typename T>
hipError_t launch_coarse(const Level<T>* Ls, const double* const* chol, int n, int nslots, hipStream_t st);
// Thomas factors of the lines along `dir` of one level (L: host copy of its descriptor)
template <typename T>
hipError_t launch_line_factor(const Level<T>& L, int dir, hipStream_t st);
// allows the cyclic-reduction line kernels their LDS (once per process)
template <typename T>
hipError_t prepare_line_cr();
// one line-smoothing op (arg from line_arg) on level s of every slot: cyclic
// reduction in LDS, one workgroup per line, or one thread per line (Thomas,
// factors from setup) for lines too long for LDS
template <typename T>
hipError_t launch_line(const Level<T>* Ls, const LevelShape& s, int arg, T omega, int kind, int nslots,
                       hipStream_t st);
template <typename T>
hipError_t launch_subcycle(const Level<T>* levs, int nlev, const DOp* prog, const int* beg, const int* cnt,
                           const double* const* chol, int ncu, T omega, int ncol, int nslots, hipStream_t st);
template <typename T>
hipError_t launch_resnorm(const Level<T>* Ls, const LevelShape& s, int mode, T* rout, const Level<float>* R32s,
                          int kind, bool oned, int nslots, hipStream_t st);

template <typename T>
hipError_t prepare_subcycle_lds();
template <typename T>
hipError_t launch_subcycle_lds(const Level<T>* levs, int nlev, int top, const DOp* prog, const int* beg,
                               const int* cnt, const double* const* chol, int ncu, T omega, int ncol, int narr,
                               int kind, bool oned, size_t lds_bytes, int nslots, hipStream_t st);

template <typename T>
hipError_t launch_norm_finish(const Level<T>* Ls, int nblocks, int mode, int nslots, hipStream_t st);

int norm_blocks(const LevelShape& s);

hipError_t launch_outer_update(const Level<double>* L64, const Level<float>* L32, const LevelShape& s, int nslots,
                               hipStream_t st);
hipError_t launch_zero_boundary(double* x, int nx, int ny, int pitch, int py, hipStream_t st);
// cell coefficients of a refined grid in the equidistant form (kx ry/rx, ky rx/ry)
hipError_t launch_graded_cells(const double* kx, const double* ky, int in_oned, const double* rx, const double* ry,
                               double* kxo, double* kyo, int ncx, int nrows, hipStream_t st);
hipError_t launch_q1_bands(double* band, int bstride, int bpitch, int nrows, int nx, int ny, int py, const double* kx,
                           const double* ky, int kpitch, double hx, double hy, hipStream_t st);
hipError_t launch_rap(double* cband, int cbstride, int cbpitch, int cnrows, int ncx, int ncy, const double* fband,
                      int fbstride, int fbpitch, int nxf, int nyf, int py, hipStream_t st);
hipError_t launch_dense_coarse(double* A, int n, int nx, int ny, int py, int kind, double cx, double cy, double dg,
                               const double* band, int bstride, int bpitch, hipStream_t st);
hipError_t launch_cholesky(double* A, int n, int* info, hipStream_t st);
// X = A^-1 (n x n) from the Cholesky factor of A
hipError_t launch_chol_inverse(const double* Lf, double* X, int n, hipStream_t st);
hipError_t launch_count_bad(const double* v, long n, int* count, hipStream_t st);
hipError_t launch_count_nonfinite(const double* v, int nx, int ny, int pitch, int py, int* count, hipStream_t st);
hipError_t launch_to_float(const double* s, float* d, long n, hipStream_t st);
// band D (index BAND_D) = 1 / band C of a level's band storage
hipError_t launch_inv_diag(double* band, int bstride, hipStream_t st);
hipError_t launch_coeff_grad(const double* u, const double* lam, double* g, int nx, int ny, int py, double hx,
                             double hy, hipStream_t st);

}  // namespace mg
