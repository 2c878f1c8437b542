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

// Output tile TX x TY (both even), halo H, and the tile grid of a level.
// wide: the region is wide_width() columns (TX = wide_width() - 2 H) in the
// parity-split LDS layout of the wide-tile kernels.
struct TileGeom {
  int TX, TY, H, ntx, nty, wide;
};

TileGeom tile_geom(int nx, int ny, int TX, int TY, int H);
TileGeom wide_geom(int nx, int ny, int TY, int H);
int wide_width();

template <typename T>
size_t pre_lds_bytes(const TileGeom& g, int ncol);
template <typename T>
size_t post_lds_bytes(const TileGeom& g, int ncol);
template <typename T>
hipError_t prepare_fused();
template <typename T>
hipError_t launch_pre(const Level<T>* Fs, const Level<T>* Cs, const TileGeom& g, int nsteps, int ncol, T omega,
                      int kind, bool oned, bool fine, int nslots, hipStream_t st, bool zero_x = false);
template <typename T>
hipError_t launch_post(const Level<T>* Fs, const Level<T>* Cs, const TileGeom& g, int nsteps, int ncol, T omega,
                       int mode, const Level<double>* X64s, int kind, bool oned, bool fine, int nslots,
                       hipStream_t st, bool with_finish = true);

}  // namespace mg
