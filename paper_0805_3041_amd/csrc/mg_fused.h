// Host-visible launchers of the fused, LDS-tiled level passes (mg_fused.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "mg_kernels.h"

namespace mg {

constexpr size_t FUSED_LDS_MAX = 150 * 1024;
constexpr size_t WIDE_LDS_TARGET = 78 * 1024;  // two wide-tile workgroups per CU (160 KB)

// POST_MIXED_KEEP: as POST_MIXED without writing e = 0 (wide tiles; the
// next finest pre-pass starts from e = 0 without reading e).
enum PostMode { POST_PLAIN = 0, POST_NORM = 1, POST_MIXED = 2, POST_MIXED_KEEP = 3 };

// Start of a pre-pass (wide tiles): load x and b (PRE_LOAD); take x = 0
// without reading it (PRE_ZERO); on the FP32 finest level of the mixed
// form, also form the right-hand side r = b - A x from the FP64 level in
// the pass itself, with the partial sums of its norm (PRE_RESID), or only
// that (PRE_RESID_ONLY: r into b and the partial sums, no smoothing).
enum PreMode { PRE_LOAD = 0, PRE_ZERO = 1, PRE_RESID = 2, PRE_RESID_ONLY = 3 };

// Output tile TX x TY (both even), halo H, and the tile grid of a level.
// wide: the region is wide_width() columns (TX = wide_width() - 2 H) in the
// parity-split LDS layout of the wide-tile kernels, and TY + 2 Hy rows (the
// row halo Hy is smaller than H with four colours; small tiles: Hy = H).
struct TileGeom {
  int TX, TY, H, ntx, nty, wide, Hy;
};

TileGeom tile_geom(int nx, int ny, int TX, int TY, int H);
TileGeom wide_geom(int nx, int ny, int TY, int H, int Hy);
int wide_width();

template <typename T>
size_t pre_lds_bytes(const TileGeom& g, int ncol);
template <typename T>
size_t post_lds_bytes(const TileGeom& g, int ncol);
template <typename T>
hipError_t prepare_fused();
// Whether the residual modes fit a pre-pass tile (its region rows are held
// per wave in registers), and the operator (5-point, or 9-point with
// coefficients constant along y).
bool pre_resid_fits(const TileGeom& g);
bool pre_resid_kind(int kind, bool oned);
template <typename T>
hipError_t launch_pre(const Level<T>* Fs, const Level<T>* Cs, const TileGeom& g, int nsteps, int ncol, T omega,
                      int kind, bool oned, bool fine, int nslots, hipStream_t st, int mode = PRE_LOAD,
                      const Level<double>* X64s = nullptr);
template <typename T>
hipError_t launch_post(const Level<T>* Fs, const Level<T>* Cs, const TileGeom& g, int nsteps, int ncol, T omega,
                       int mode, const Level<double>* X64s, int kind, bool oned, bool fine, int nslots,
                       hipStream_t st, bool with_finish = true);

}  // namespace mg
