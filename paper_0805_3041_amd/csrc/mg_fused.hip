// Fused, LDS-tiled passes of one level visit (temporal blocking).
//
// Pre-pass : nu1 smoothing steps, defect, full-weighting restriction.
//            reads x (Level::x) and b, writes the smoothed iterate to the
//            ping-pong buffer Level::t, the coarse right-hand side and a zero
//            coarse start vector.
// Post-pass: bilinear prolongation of the coarse correction, nu2 smoothing
//            steps; reads Level::t, b and the coarse x, writes Level::x.
//            On the finest level it can also compute the residual norm of the
//            new iterate (the stopping test) or, in the mixed-precision form,
//            add the FP32 correction into the FP64 iterate.
//
// Each workgroup owns an output tile of TX x TY nodes and loads a region
// widened by a halo of H nodes.  Every Gauss-Seidel colour sweep (or Jacobi
// step) is valid on a region one node narrower than the previous one, so
// after the k-th sweep the nodes at distance >= k from the region's edge hold
// exactly the values a sweep over the whole grid would give: the arithmetic
// per node is the shared device function of mg_device.h.  Reading x and
// writing the result to different buffers keeps workgroups from seeing a
// neighbour's already-updated nodes in their halo.
//
// Cost model: the passes are bound by instruction issue, not by HBM, so the
// per-node work is kept small: a tile whose region lies inside the grid's
// unknowns (all but the tiles along a Dirichlet edge) runs a sweep body with
// no boundary tests; node positions advance incrementally instead of being
// divided out of a flat index; 9-point operators whose coefficients vary
// along x only keep the tile's columns of their bands in LDS.
#include <type_traits>

#include "mg_fused.h"

namespace mg {

constexpr int FT = 512;  // threads per tile workgroup

struct TileMap {
  int i0, j0, H, nx, ny, py;
  __device__ __forceinline__ int gi(int li) const { return i0 - H + li; }
  __device__ __forceinline__ int gj(int lj) const { return j0 - H + lj; }  // not wrapped
  __device__ __forceinline__ bool unknown(int i, int j) const {
    const bool in_i = (unsigned)(i - 1) < (unsigned)(nx - 2);
    return py ? in_i : (in_i && (unsigned)(j - 1) < (unsigned)(ny - 2));
  }
  // stored row of global row j (periodic y wraps; a region may overhang
  // by more than one period on small coarse levels)
  __device__ __forceinline__ int wrapj(int j) const {
    if (py) {
      while (j < 0) j += ny;
      while (j >= ny) j -= ny;
    }
    return j;
  }
};

// Solve-finished flag of a tile kernel's problem, batched launches: tested at
// once (most slots are finished in most cycles).  Its own branch, so that a
// one-problem launch never waits on the flag before issuing its loads; that
// launch reads the flag after its region loads and tests it at the first
// barrier (a finished problem's kernels store nothing).
__device__ __forceinline__ bool batched_done(const SolveState* st) {
  if (gridDim.z > 1) return st->done != 0;
  return false;
}

// Tile index -> (tx, ty).  Consecutive workgroup ids go to different XCDs
// (round-robin dispatch over 8), so ids are regrouped to give each XCD a
// contiguous band of tiles: its L2 then holds the band across passes.
__device__ __forceinline__ void tile_coords(int ntx, int nty, int& tx, int& ty) {
  const int nt = ntx * nty;
  const int b = blockIdx.x;
  int t = b;
  const int per = nt / 8;
  if (per > 0 && b < per * 8) t = (b & 7) * per + (b >> 3);
  ty = t / ntx;
  tx = t - ty * ntx;
}

// Row-major walk over an index space with nk columns: a thread visits
// idx, idx + FT, idx + 2 FT, ... and keeps (row r, column k) up to date
// with adds instead of a division per step.
struct Walk {
  int r, k, dq, dk, nk;
  __device__ __forceinline__ Walk(int idx, int nk_) : nk(nk_) {
    const FDiv d(nk_);
    r = d.q(idx);
    k = idx - r * nk_;
    dq = d.q(FT);
    dk = FT - dq * nk_;
  }
  __device__ __forceinline__ void next() {
    k += dk;
    r += dq;
    if (k >= nk) {
      k -= nk;
      ++r;
    }
  }
};

// Coefficients of the node at tile column li (global gi, wrapped row gjw).
// B1: the bands vary along x only and the tile's W columns of each band sit
// in LDS (band k at bl + k W), giving the same values as coefs().
template <typename T, int K, bool B1>
__device__ __forceinline__ Cf<T> tcoef(const Level<T>& L, const MG_LDS T* bl, int W, int li, int gi, int gjw) {
  if constexpr (K == ST5) {
    return Cf<T>{};
  } else if constexpr (B1) {
    const MG_LDS T* p = bl + li;
    Cf<T> c;
    c.C = p[0];
    c.Ep = p[W];
    c.Ew = p[W - 1];
    c.Np = p[2 * W];
    c.Ns = c.Np;
    c.NEp = p[3 * W];
    c.NEsw = p[3 * W - 1];
    c.NWp = p[4 * W];
    c.NWse = p[4 * W + 1];
    c.D = p[BAND_D * W];
    return c;
  } else {
    return coefs<K>(L, gi, gjw, wrap_dn(gjw, L.ny, L.py));
  }
}

// Row of a tile that does not need boundary tests (EDGE false): the global
// row, wrapped once for periodic y (the region is at most one period tall).
__device__ __forceinline__ int wrap_once(int j, int ny, int py) {
  if (!py) return j;
  return j < 0 ? j + ny : (j >= ny ? j - ny : j);
}

// One Gauss-Seidel colour sweep over the region shrunk by s.
// NCOL 4: colour c holds i = c & 1, j = c >> 1 (mod 2); NCOL 2: colour c
// holds (i + j) mod 2 == c.  Parities are those of global indices.
template <typename T, int K, int NCOL, bool B1, bool EDGE>
__device__ void sweep_colour(const Level<T>& L, const TileMap& m, MG_LDS T* x, const MG_LDS T* b,
                             const MG_LDS T* bl, int W, int R, int s, int c, T omega) {
  constexpr int NB = nbatch(K);
  const int hiW = W - s, hiR = R - s;
  int li0 = s, lj0 = s, rs = 1, nk, nr, par = 0;
  if constexpr (NCOL == 4) {
    li0 = s + ((m.gi(s) ^ c) & 1);
    lj0 = s + ((m.gj(s) ^ (c >> 1)) & 1);
    nk = li0 < hiW ? (hiW - li0 + 1) >> 1 : 0;
    nr = lj0 < hiR ? (hiR - lj0 + 1) >> 1 : 0;
    rs = 2;
  } else {
    nk = (hiW - s + 1) >> 1;
    nr = hiR - s;
    par = (m.gi(s) + m.gj(s) + c) & 1;  // column offset of the colour in row r: (par + r) & 1
  }
  const int n = nr * nk;
  if (n <= 0) return;
  Walk w(threadIdx.x, nk);
  for (int base = threadIdx.x; base < n; base += FT * NB) {
    int pos[NB], li[NB], gi[NB], gjw[NB];
    bool ok[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int lj = lj0 + rs * w.r;
      int l = li0 + 2 * w.k;
      if constexpr (NCOL == 2) l += (par + w.r) & 1;
      ok[u] = base + u * FT < n && l < hiW;
      w.next();
      li[u] = l;
      pos[u] = lj * W + l;
      gi[u] = m.gi(l);
      gjw[u] = 0;
      if constexpr (EDGE) {
        const int gj = m.gj(lj);
        ok[u] = ok[u] && m.unknown(gi[u], gj);
        if (ok[u] && K == ST9 && !B1) gjw[u] = m.wrapj(gj);
      } else if constexpr (K == ST9 && !B1) {
        gjw[u] = wrap_once(m.gj(lj), m.ny, m.py);
      }
    }
    Nbr<T> v[NB];
    Cf<T> a[NB];
    T bp[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (!ok[u]) continue;
      v[u] = gather<K>(L, LXW<T>{x + pos[u], W}, false);
      bp[u] = b[pos[u]];
      a[u] = tcoef<T, K, B1>(L, bl, W, li[u], gi[u], gjw[u]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (ok[u]) x[pos[u]] = sor_v(gs_v<K>(L, a[u], v[u], bp[u]), x + pos[u], omega);
  }
}

// Every node of the region shrunk by s, NB nodes per thread per round
// (their loads issued before any store).  JACOBI: damped Jacobi step
// src -> dst.  Otherwise the defect b - A src, written in place into b (a
// node's defect reads only its own b), 0 at nodes that are not unknowns.
template <typename T, int K, bool B1, bool EDGE, bool JACOBI>
__device__ void sweep_region(const Level<T>& L, const TileMap& m, const MG_LDS T* src, MG_LDS T* dst,
                             MG_LDS T* b, const MG_LDS T* bl, int W, int R, int s, T omega) {
  constexpr int NB = nbatch(K);
  const int cols = W - 2 * s, n = (R - 2 * s) * cols;
  if (n <= 0) return;
  Walk w(threadIdx.x, cols);
  for (int base = threadIdx.x; base < n; base += FT * NB) {
    int pos[NB], li[NB], gi[NB], gjw[NB];
    bool ok[NB], in[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int lj = s + w.r, l = s + w.k;
      in[u] = base + u * FT < n;
      ok[u] = in[u];
      w.next();
      li[u] = l;
      pos[u] = lj * W + l;
      gi[u] = m.gi(l);
      gjw[u] = 0;
      if constexpr (EDGE) {
        const int gj = m.gj(lj);
        ok[u] = ok[u] && m.unknown(gi[u], gj);
        if (ok[u] && K == ST9 && !B1) gjw[u] = m.wrapj(gj);
      } else if constexpr (K == ST9 && !B1) {
        gjw[u] = wrap_once(m.gj(lj), m.ny, m.py);
      }
    }
    Nbr<T> v[NB];
    Cf<T> a[NB];
    T bp[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (!ok[u]) continue;
      v[u] = gather<K>(L, LXW<T>{src + pos[u], W}, true);
      bp[u] = b[pos[u]];
      a[u] = tcoef<T, K, B1>(L, bl, W, li[u], gi[u], gjw[u]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if constexpr (JACOBI) {
        if (ok[u]) dst[pos[u]] = jac_v<K>(L, a[u], v[u], bp[u], omega);
      } else {
        if (in[u]) b[pos[u]] = ok[u] ? defect_v<K>(L, a[u], v[u], bp[u]) : (T)0;
      }
    }
  }
}

// nsteps smoothing steps on the region; returns the LDS array holding the
// result (x, or t after an odd number of Jacobi steps).
template <typename T, int K, int NCOL, bool B1, bool EDGE>
__device__ MG_LDS T* tile_smooth(const Level<T>& L, const TileMap& m, MG_LDS T* x, MG_LDS T* t, MG_LDS T* b,
                                 const MG_LDS T* bl, int W, int R, int nsteps, T omega) {
  int s = 1;
  if constexpr (NCOL == 0) {
    MG_LDS T* src = x;
    MG_LDS T* dst = t;
    for (int k = 0; k < nsteps; ++k, ++s) {
      sweep_region<T, K, B1, EDGE, true>(L, m, src, dst, b, bl, W, R, s, omega);
      __syncthreads();
      MG_LDS T* tmp = src;
      src = dst;
      dst = tmp;
    }
    return src;
  } else {
    for (int k = 0; k < nsteps; ++k) {
      for (int c = 0; c < NCOL; ++c, ++s) {
        sweep_colour<T, K, NCOL, B1, EDGE>(L, m, x, b, bl, W, R, s, c, omega);
        __syncthreads();
      }
    }
    return x;
  }
}

// False when every node of the region shrunk by 1 is an unknown and (for
// 9-point operators read from 2-D global bands on a periodic level) the
// region is at most one period tall, so a sweep body needs no boundary
// tests.  Uniform over the workgroup.
template <typename T, int K, bool B1>
__device__ __forceinline__ bool tile_edge(const Level<T>& F, const TileMap& m, int W, int R) {
  const bool in_i = m.gi(1) >= 1 && m.gi(W - 2) <= F.nx - 2;
  bool in_j;
  if (F.py)
    in_j = (K == ST9 && !B1) ? R <= F.ny : true;
  else
    in_j = m.gj(1) >= 1 && m.gj(R - 2) <= F.ny - 2;
  return !(in_i && in_j);
}

// The tile's W columns of the NBANDS bands of a level whose bands vary
// along x only.  Columns outside the grid are clamped (no unknown reads
// them: an unknown's columns i-1 .. i+1 lie inside).
template <typename T>
__device__ void load_bands(const Level<T>& F, const TileMap& m, MG_LDS T* dst, int W) {
  for (int idx = threadIdx.x; idx < NBANDS * W; idx += FT) {
    const int k = idx / W, li = idx - k * W;
    const int g = min(max(m.gi(li), 0), F.nx - 1);
    dst[idx] = bandp(F, k)[g];
  }
}

__device__ __forceinline__ double wg_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < FT / 64; ++k) s += sh[k];
  __syncthreads();
  return s;
}

constexpr int LB = 4;  // region nodes a thread loads from global memory per round

// ------------------------------------------------------------------ pre-pass

template <typename T, int K, int NCOL, bool B1, bool EDGE>
__device__ __forceinline__ MG_LDS T* pre_body(const Level<T>& F, const TileMap& m, MG_LDS T* x, MG_LDS T* t,
                                              MG_LDS T* b, const MG_LDS T* bl, int W, int R, int H, int nsteps,
                                              T omega) {
  MG_LDS T* xs = tile_smooth<T, K, NCOL, B1, EDGE>(F, m, x, t, b, bl, W, R, nsteps, omega);
  // defect on the region shrunk by H - 1 (in place into b)
  sweep_region<T, K, B1, EDGE, false>(F, m, xs, nullptr, b, bl, W, R, H - 1, omega);
  return xs;
}

// FINE: instantiation used on the finest level only (a separate symbol, so
// profiles and timings of the finest pass are not mixed with coarser ones).
template <typename T, int K, bool FINE, int NCOL, bool B1>
__global__ void __launch_bounds__(FT) k_pre(const Level<T>* __restrict__ Fs, const Level<T>* __restrict__ Cs, int TX,
                                            int TY, int H, int ntx, int nty, int nsteps, T omega) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Level<T> F = Fs[blockIdx.z];
  if (batched_done(F.st)) return;
  const Level<T> C = Cs[blockIdx.z];
  int tx, ty;
  tile_coords(ntx, nty, tx, ty);
  const int W = TX + 2 * H, R = TY + 2 * H;
  MG_LDS T* x = lds_cast<T>(smem_raw);
  MG_LDS T* b = x + W * R;
  MG_LDS T* t = b + W * R;  // Jacobi only
  MG_LDS T* bl = b + W * R * (NCOL == 0 ? 2 : 1);
  const TileMap m{tx * TX, ty * TY, H, F.nx, F.ny, F.py};
  if constexpr (B1) load_bands(F, m, bl, W);

  {
    Walk w(threadIdx.x, W);
    const int n = W * R;
    for (int base = threadIdx.x; base < n; base += FT * LB) {
      T xv[LB], bv[LB];
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int gi = m.gi(w.k), gj = m.gj(w.r);
        w.next();
        xv[u] = bv[u] = (T)0;
        if (base + u * FT < n && m.unknown(gi, gj)) {
          const size_t p = (size_t)m.wrapj(gj) * F.pitch + gi;
          xv[u] = F.x[p];
          bv[u] = F.b[p];
        }
      }
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int idx = base + u * FT;
        if (idx < n) {
          x[idx] = xv[u];
          b[idx] = bv[u];
          if constexpr (NCOL == 0) t[idx] = (T)0;
        }
      }
    }
  }
  const int done = F.st->done;
  __syncthreads();
  if (done) return;

  MG_LDS T* xs;
  if (tile_edge<T, K, B1>(F, m, W, R))
    xs = pre_body<T, K, NCOL, B1, true>(F, m, x, t, b, bl, W, R, H, nsteps, omega);
  else
    xs = pre_body<T, K, NCOL, B1, false>(F, m, x, t, b, bl, W, R, H, nsteps, omega);
  __syncthreads();

  // full weighting at the coarse nodes of the tile; zero coarse start
  {
    const int ca = TX >> 1, n = ca * (TY >> 1);
    const int lo = C.py ? 0 : 1, hi = C.py ? C.ny - 1 : C.ny - 2;
    Walk w(threadIdx.x, ca);
    for (int idx = threadIdx.x; idx < n; idx += FT) {
      const int a = w.k, rb = w.r;
      w.next();
      const int I = (m.i0 >> 1) + a, J = (m.j0 >> 1) + rb;
      if (I < 1 || I > C.nx - 2 || J < lo || J > hi) continue;
      const int li = H + 2 * a, lj = H + 2 * rb;
      const MG_LDS T* d0 = b + (lj - 1) * W + li;
      const MG_LDS T* d1 = d0 + W;
      const MG_LDS T* d2 = d1 + W;
      const T g = fw_combine(fw_row(d0[-1], d0[0], d0[1]), fw_row(d1[-1], d1[0], d1[1]), fw_row(d2[-1], d2[0], d2[1]));
      const size_t q = (size_t)J * C.pitch + I;
      C.b[q] = g;
      C.x[q] = (T)0;
    }
  }
  // smoothed iterate of the output nodes -> ping-pong buffer
  {
    const int n = TX * TY;
    Walk w(threadIdx.x, TX);
    for (int idx = threadIdx.x; idx < n; idx += FT) {
      const int lj = H + w.r, li = H + w.k;
      w.next();
      const int gj = m.gj(lj), gi = m.gi(li);
      if (!m.unknown(gi, gj) || gj >= F.ny) continue;
      F.t[(size_t)gj * F.pitch + gi] = xs[lj * W + li];
    }
  }
}

// ------------------------------------------------------------------ post-pass

// mode: POST_PLAIN, POST_NORM (finest level: stopping test of the new
// iterate), POST_MIXED (finest FP32 level: x64 += e, e = 0).
template <typename T, int K, bool FINE, int NCOL, bool B1>
__global__ void __launch_bounds__(FT) k_post(const Level<T>* __restrict__ Fs, const Level<T>* __restrict__ Cs, int TX,
                                             int TY, int H, int ntx, int nty, int nsteps, T omega, int mode,
                                             const Level<double>* __restrict__ X64s) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double sh[FT / 64];
  const Level<T> F = Fs[blockIdx.z];
  SolveState* st = F.st;
  if (batched_done(st)) return;
  const Level<T> C = Cs[blockIdx.z];
  const bool wtd = F.wl != nullptr;  // adaptive omega_l
  const T wv = wtd ? *F.wl : (T)1;
  int tx, ty;
  tile_coords(ntx, nty, tx, ty);
  const int W = TX + 2 * H, R = TY + 2 * H;
  MG_LDS T* x = lds_cast<T>(smem_raw);
  MG_LDS T* b = x + W * R;
  MG_LDS T* t = b + W * R;
  const TileMap m{tx * TX, ty * TY, H, F.nx, F.ny, F.py};

  // coarse correction covering the region
  const int cI0 = m.gi(0) >> 1, cJ0 = m.gj(0) >> 1;
  const int CW = (W >> 1) + 2, CR = (R >> 1) + 2;
  MG_LDS T* ec = t + (NCOL == 0 ? W * R : 0);
  MG_LDS T* bl = ec + CW * CR;
  if constexpr (B1) load_bands(F, m, bl, W);
  {
    const int clo = C.py ? 0 : 1, chi = C.py ? C.ny - 1 : C.ny - 2;
    const int n = CW * CR;
    Walk w(threadIdx.x, CW);
    for (int base = threadIdx.x; base < n; base += FT * LB) {
      T v[LB];
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int I = cI0 + w.k;
        int J = cJ0 + w.r;
        w.next();
        v[u] = (T)0;
        if (C.py) {
          while (J < 0) J += C.ny;
          while (J >= C.ny) J -= C.ny;
        }
        if (base + u * FT < n && I >= 1 && I <= C.nx - 2 && J >= clo && J <= chi) v[u] = C.x[(size_t)J * C.pitch + I];
      }
#pragma unroll
      for (int u = 0; u < LB; ++u)
        if (base + u * FT < n) ec[base + u * FT] = v[u];
    }
  }
  __syncthreads();
  {
    Walk w(threadIdx.x, W);
    const int n = W * R;
    for (int base = threadIdx.x; base < n; base += FT * LB) {
      T tv[LB], bv[LB];
      int gi[LB], gj[LB];
      bool ok[LB];
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        gi[u] = m.gi(w.k);
        gj[u] = m.gj(w.r);
        w.next();
        tv[u] = bv[u] = (T)0;
        ok[u] = base + u * FT < n && m.unknown(gi[u], gj[u]);
        if (ok[u]) {
          const size_t p = (size_t)m.wrapj(gj[u]) * F.pitch + gi[u];
          tv[u] = F.t[p];
          bv[u] = F.b[p];
        }
      }
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int idx = base + u * FT;
        if (idx >= n) continue;
        T xv = (T)0;
        if (ok[u]) {
          const int I = gi[u] >> 1, J = gj[u] >> 1;
          const MG_LDS T* r0 = ec + (J - cJ0) * CW + (I - cI0);
          const MG_LDS T* r1 = r0 + CW;
          xv = add_correction(tv[u], prolong_combine(r0[0], r0[1], r1[0], r1[1], gi[u] & 1, gj[u] & 1), wtd, wv);
        }
        x[idx] = xv;
        b[idx] = bv[u];
        if constexpr (NCOL == 0) t[idx] = (T)0;
      }
    }
  }
  const int done = F.st->done;
  __syncthreads();
  if (done) return;

  MG_LDS T* xs;
  if (tile_edge<T, K, B1>(F, m, W, R))
    xs = tile_smooth<T, K, NCOL, B1, true>(F, m, x, t, b, bl, W, R, nsteps, omega);
  else
    xs = tile_smooth<T, K, NCOL, B1, false>(F, m, x, t, b, bl, W, R, nsteps, omega);

  double acc = 0.0;
  const int n = TX * TY;
  Walk w(threadIdx.x, TX);
  for (int idx = threadIdx.x; idx < n; idx += FT) {
    const int lj = H + w.r, li = H + w.k;
    w.next();
    const int gj = m.gj(lj), gi = m.gi(li);
    if (!m.unknown(gi, gj) || gj >= F.ny) continue;
    const size_t p = (size_t)gj * F.pitch + gi;
    const int q = lj * W + li;
    if (mode == POST_MIXED || mode == POST_MIXED_KEEP) {
      const Level<double>& X = X64s[blockIdx.z];
      X.x[(size_t)gj * X.pitch + gi] += (double)xs[q];
      F.x[p] = (T)0;
    } else {
      F.x[p] = xs[q];
      if (mode == POST_NORM) {
        const T d = defect_v<K>(F, tcoef<T, K, B1>(F, bl, W, li, gi, gj), gather<K>(F, LXW<T>{xs + q, W}, true), b[q]);
        acc += (double)d * (double)d;
      }
    }
  }
  if ((mode == POST_MIXED || mode == POST_MIXED_KEEP) && blockIdx.x == 0 && threadIdx.x == 0) st->pending = 1;
  if (mode == POST_NORM) {
    const double part = wg_sum(acc, sh);
    if (threadIdx.x == 0) st->partial[blockIdx.x] = part;
  }
}

// ------------------------------------------------------------------ wide tiles
//
// Variant for large levels.  The region is WW = 128 columns wide (output
// width TX = WW - 2H) and TY + 2Hy rows tall (row halo Hy: see
// wrow_shrink), and each LDS row holds the arrays side by side, every
// array split by column parity:
//   [x even | x odd | b even | b odd (| t even | t odd)],  WH = 64 per half.
// A colour sweep updates one column parity, so lane l owns the column of
// half-index A = A0 + l (unit stride in LDS, no bank conflicts) for the
// whole sweep and each wave takes whole rows (row indices are uniform).
// All stencil reads of a node then sit at compile-time offsets from one
// address, and per-column quantities (bands that vary along x only, the
// column's boundary test) are computed once per sweep instead of per node.

constexpr int WW = 128;
constexpr int WH = WW / 2;
constexpr int NWAVE = FT / 64;
constexpr int UL = 4;  // rows whose global loads a wave issues before its first wait
constexpr int ULR = 8;  // region rows a wave loads per round in the wide passes (one round up to 64 rows)

template <int NCOL>
constexpr int wide_narr() {
  return NCOL == 0 ? 3 : 2;
}

struct WMap {
  int i0, j0, H, Hy, nx, ny, py;  // column halo H, row halo Hy
  __device__ __forceinline__ int gi(int li) const { return i0 - H + li; }
  __device__ __forceinline__ int gj(int lj) const { return j0 - Hy + lj; }
  __device__ __forceinline__ bool col_ok(int li) const { return (unsigned)(gi(li) - 1) < (unsigned)(nx - 2); }
  __device__ __forceinline__ bool row_ok(int lj) const {
    return py ? true : (unsigned)(gj(lj) - 1) < (unsigned)(ny - 2);
  }
  __device__ __forceinline__ int wrapj(int j) const {
    if (py) {
      while (j < 0) j += ny;
      while (j >= ny) j -= ny;
    }
    return j;
  }
};

// Offset of column li inside an array's row (parity split).
__device__ __forceinline__ int wcol(int li) { return (li & 1) * WH + (li >> 1); }

// x around a node of column parity Q: p points at row lj - 1, half-index A
// of the array (p = array + (lj - 1) P + A).  The node's own column is at
// `own`, its west and east neighbours in the other half at ow, ow + 1.
template <typename T, int K, int P, int Q, bool CENTRE>
__device__ __forceinline__ Nbr<T> wgather(const MG_LDS T* p) {
  constexpr int own = Q ? WH : 0, ow = Q ? 0 : WH - 1;
  Nbr<T> v{};
  v.s = p[own];
  v.w = p[P + ow];
  v.e = p[P + ow + 1];
  if (CENTRE) v.c = p[P + own];
  v.n = p[2 * P + own];
  if (K != ST5) {
    v.sw = p[ow];
    v.se = p[ow + 1];
    v.nw = p[2 * P + ow];
    v.ne = p[2 * P + ow + 1];
  }
  return v;
}

// Coefficients of column half-index A (parity Q) from the LDS copy of
// bands that vary along x only (band k at bl + k WW, parity split).
template <typename T, int Q>
__device__ __forceinline__ Cf<T> wcoef_cols(const MG_LDS T* bl, int A) {
  constexpr int own = Q ? WH : 0, oth = Q ? 0 : WH;
  const MG_LDS T* p = bl + A;
  Cf<T> c;
  c.C = p[own];
  c.Ep = p[WW + own];
  c.Ew = p[WW + oth - 1 + Q];
  c.Np = p[2 * WW + own];
  c.Ns = c.Np;
  c.NEp = p[3 * WW + own];
  c.NEsw = p[3 * WW + oth - 1 + Q];
  c.NWp = p[4 * WW + own];
  c.NWse = p[4 * WW + oth + Q];
  c.D = p[BAND_D * WW + own];
  return c;
}

// Coefficients of node (gi, row lj) for a sweep: hoisted column values
// (B1), from global memory (2-D: the four cells of a finest level that
// keeps them, which stay in L2 across the sweeps of a pass, else the six
// bands), or none (5-point).
template <typename T, int K, bool B1>
__device__ __forceinline__ Cf<T> wcoef(const Level<T>& L, const WMap& m, const Cf<T>& col, int gi, int lj) {
  if constexpr (K == ST5 || B1) {
    return col;
  } else {
    const int gjw = m.wrapj(m.gj(lj));
    return coefs<K>(L, gi, gjw, wrap_dn(gjw, L.ny, L.py));
  }
}

// Wave index as a scalar: row loops then run on the scalar unit.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Gauss-Seidel update of the column-parity-Q nodes of a colour on the rows
// lj0 + rstep (wave + NWAVE k) < hiR that carry unknowns (a contiguous range
// of local rows, found once), two rows per round.  Loads are issued for every
// lane (addresses stay inside the region's rows); only lanes whose column is
// an unknown of the colour store.  SOR: relaxation factor != 1 (a plain
// Gauss-Seidel sweep then has no per-node test).
template <typename T, int K, int NCOL, bool B1, int Q, bool SOR>
__device__ void wcolour_rows(const Level<T>& L, const WMap& m, MG_LDS T* lds, const Cf<T>& col, int hiR, int lj0,
                             int rstep, int A, bool lane_ok, int gi, T omega) {
  constexpr int P = wide_narr<NCOL>() * WW;
  constexpr int own = Q ? WH : 0;
  const int step = rstep * NWAVE;
  auto node = [&](int lj) -> T {
    const Nbr<T> v = wgather<T, K, P, Q, false>(lds + (lj - 1) * P + A);
    const T gs = gs_v<K>(L, wcoef<T, K, B1>(L, m, col, gi, lj), v, lds[lj * P + WW + own + A]);
    if constexpr (SOR) {
      return sor_v(gs, lds + lj * P + own + A, omega);
    } else {
      return gs;
    }
  };
  int lj = lj0 + rstep * wave_id();
  int end = hiR;
  if (!m.py) {  // rows of unknowns: 1 <= global row <= ny - 2
    const int lo = 1 - m.j0 + m.Hy, hi = m.ny - 1 - m.j0 + m.Hy;
    if (lj < lo) lj += (lo - lj + step - 1) / step * step;
    end = min(end, hi);
  }
  for (; lj + step < end; lj += 2 * step) {
    const int lj2 = lj + step;
    const T x1 = node(lj), x2 = node(lj2);
    if (lane_ok) {
      lds[lj * P + own + A] = x1;
      lds[lj2 * P + own + A] = x2;
    }
  }
  if (lj < end) {
    const T x1 = node(lj);
    if (lane_ok) lds[lj * P + own + A] = x1;
  }
}

// Lane plan of a pass's colour sweeps: lane l owns column q + 2 l of each
// local column parity q for every sweep (half-index A = l), so whether the
// column is an unknown, its global index and (1-D bands) its coefficients
// are found once per pass; a sweep only masks the columns outside the
// region shrunk by s.  A lane outside the unknowns still loads (its results
// are not stored), at an interior column for global band reads.
template <typename T>
struct WLanes {
  bool ok[2];
  int gi[2];
  Cf<T> col[2];
};

template <typename T, int K, bool B1>
__device__ __forceinline__ WLanes<T> wlanes(const WMap& m, const MG_LDS T* bl) {
  const int lane = threadIdx.x & 63;
  WLanes<T> w;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int li = q + 2 * lane;
    w.ok[q] = m.col_ok(li);
    w.gi[q] = w.ok[q] ? m.gi(li) : 1;
    w.col[q] = Cf<T>{};
  }
  if constexpr (K == ST9 && B1) {
    w.col[0] = wcoef_cols<T, 0>(bl, lane);
    w.col[1] = wcoef_cols<T, 1>(bl, lane);
  }
  return w;
}

// One Gauss-Seidel colour sweep over the region shrunk by s columns and sr
// rows (colours as in sweep_colour; i0, j0 are even, so local and global
// parities agree up to H and Hy).
template <typename T, int K, int NCOL, bool B1>
__device__ void wsweep_colour(const Level<T>& L, const WMap& m, MG_LDS T* lds, const WLanes<T>& w, int R, int s,
                              int sr, int c, T omega) {
  const int wave = wave_id(), lane = threadIdx.x & 63;
  int q, lj0, rstep;
  if constexpr (NCOL == 4) {
    const int qr = ((c >> 1) + m.Hy) & 1;
    lj0 = sr + ((sr ^ qr) & 1);
    rstep = 2;
    q = ((c & 1) + m.H) & 1;
  } else {
    // the wave's rows s + wave + NWAVE k share the parity of s + wave
    // (two colours: rows and columns shrink alike, sr = s, Hy = H)
    lj0 = sr;
    rstep = 1;
    q = (c + sr + wave) & 1;
  }
  const int li = q + 2 * lane;
  if (omega == (T)1) {
    if (q)
      wcolour_rows<T, K, NCOL, B1, 1, false>(L, m, lds, w.col[1], R - sr, lj0, rstep, lane,
                                             w.ok[1] && li >= s && li < WW - s, w.gi[1], omega);
    else
      wcolour_rows<T, K, NCOL, B1, 0, false>(L, m, lds, w.col[0], R - sr, lj0, rstep, lane,
                                             w.ok[0] && li >= s && li < WW - s, w.gi[0], omega);
  } else {
    if (q)
      wcolour_rows<T, K, NCOL, B1, 1, true>(L, m, lds, w.col[1], R - sr, lj0, rstep, lane,
                                            w.ok[1] && li >= s && li < WW - s, w.gi[1], omega);
    else
      wcolour_rows<T, K, NCOL, B1, 0, true>(L, m, lds, w.col[0], R - sr, lj0, rstep, lane,
                                            w.ok[0] && li >= s && li < WW - s, w.gi[0], omega);
  }
}

// Every node of the region shrunk by s columns and sr rows, both column
// parities per lane and row.  DST == 1: defect b - A src in place into b (0
// at region nodes that are not unknowns).  Otherwise damped Jacobi src ->
// dst.  Array indices: 0 x, 1 b, 2 t.
template <typename T, int K, int NCOL, bool B1, int SRC, int DST>
__device__ void wsweep_region(const Level<T>& L, const WMap& m, MG_LDS T* lds, const MG_LDS T* bl, int R, int s,
                              int sr, T omega) {
  constexpr int P = wide_narr<NCOL>() * WW;
  const int lane = threadIdx.x & 63;
  const int li0 = 2 * (((s + 1) >> 1) + lane), li1 = 2 * ((s >> 1) + lane) + 1;
  const int A0 = li0 >> 1, A1 = li1 >> 1;
  const bool in0 = li0 < WW - s, in1 = li1 < WW - s;
  const bool ok0 = in0 && m.col_ok(li0), ok1 = in1 && m.col_ok(li1);
  const int g0 = ok0 ? m.gi(li0) : 1, g1 = ok1 ? m.gi(li1) : 1;  // interior column for lanes that only load
  Cf<T> c0{}, c1{};
  if constexpr (K == ST9 && B1) {
    if (ok0) c0 = wcoef_cols<T, 0>(bl, A0);
    if (ok1) c1 = wcoef_cols<T, 1>(bl, A1);
  }
  for (int lj = sr + wave_id(); lj < R - sr; lj += NWAVE) {
    MG_LDS T* row = lds + lj * P;
    if (!m.row_ok(lj)) {
      if constexpr (DST == 1) {
        if (in0) row[WW + A0] = (T)0;
        if (in1) row[WW + WH + A1] = (T)0;
      }
      continue;
    }
    const MG_LDS T* src = lds + SRC * WW + (lj - 1) * P;
    const Nbr<T> v0 = wgather<T, K, P, 0, true>(src + A0);
    const Nbr<T> v1 = wgather<T, K, P, 1, true>(src + A1);
    const T b0 = row[WW + A0], b1 = row[WW + WH + A1];
    const Cf<T> a0 = wcoef<T, K, B1>(L, m, c0, g0, lj), a1 = wcoef<T, K, B1>(L, m, c1, g1, lj);
    if constexpr (DST == 1) {
      const T d0 = defect_v<K>(L, a0, v0, b0), d1 = defect_v<K>(L, a1, v1, b1);
      if (in0) row[WW + A0] = ok0 ? d0 : (T)0;
      if (in1) row[WW + WH + A1] = ok1 ? d1 : (T)0;
    } else {
      const T y0 = jac_v<K>(L, a0, v0, b0, omega), y1 = jac_v<K>(L, a1, v1, b1, omega);
      if (ok0) row[DST * WW + A0] = y0;
      if (ok1) row[DST * WW + WH + A1] = y1;
    }
  }
}

// Rows of the region that may be stale after s colour steps.  A colour step
// leaves stale the nodes it updates next to stale ones.  With four colours
// the column parity alternates from step to step, so stale columns advance
// one per step, but the row parity changes every second step only, so stale
// rows advance at most one per two steps: (s + 1) / 2 after s steps (the
// row halo Hy is that many rows for the sweeps, plus the defect and
// restriction rows).  Other smoothers: one per step in both directions.
template <int NCOL>
__device__ __forceinline__ int wrow_shrink(int s) {
  return NCOL == 4 ? (s + 1) >> 1 : s;
}

// nsteps smoothing steps; returns the array index (0 x, 2 t) of the result.
template <typename T, int K, int NCOL, bool B1>
__device__ int wsmooth(const Level<T>& L, const WMap& m, MG_LDS T* lds, const MG_LDS T* bl, int R, int nsteps,
                       T omega) {
  if constexpr (NCOL == 0) {
    for (int k = 0; k < nsteps; ++k) {
      if (k & 1)
        wsweep_region<T, K, NCOL, B1, 2, 0>(L, m, lds, bl, R, k + 1, k + 1, omega);
      else
        wsweep_region<T, K, NCOL, B1, 0, 2>(L, m, lds, bl, R, k + 1, k + 1, omega);
      __syncthreads();
    }
    return (nsteps & 1) ? 2 : 0;
  } else {
    const WLanes<T> w = wlanes<T, K, B1>(m, bl);
    int s = 1;
    for (int k = 0; k < nsteps; ++k)
      for (int c = 0; c < NCOL; ++c, ++s) {
        wsweep_colour<T, K, NCOL, B1>(L, m, lds, w, R, s, wrow_shrink<NCOL>(s), c, omega);
        __syncthreads();
      }
    return 0;
  }
}

// Bands that vary along x only, at the region's columns (clamped to the
// grid): fetched into registers (each thread at most two values) together
// with a kernel's other first loads, stored to LDS after them.
static_assert(NBANDS * WW >= FT && NBANDS * WW <= 2 * FT, "band fetch covers NBANDS * WW with two rounds");
template <typename T>
struct WBands {
  T v0, v1;
};
template <typename T>
__device__ __forceinline__ WBands<T> wfetch_bands(const Level<T>& F, const WMap& m) {
  WBands<T> r{(T)0, (T)0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int idx = threadIdx.x + h * FT;
    if (idx < NBANDS * WW) {
      const int k = idx / WW, li = idx - k * WW;
      const int g = min(max(m.gi(li), 0), F.nx - 1);
      (h ? r.v1 : r.v0) = bandp(F, k)[g];
    }
  }
  return r;
}
template <typename T>
__device__ __forceinline__ void wstore_bands(MG_LDS T* bl, const WBands<T>& r) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int idx = threadIdx.x + h * FT;
    if (idx < NBANDS * WW) {
      const int k = idx / WW, li = idx - k * WW;
      bl[k * WW + wcol(li)] = h ? r.v1 : r.v0;
    }
  }
}

// Residual of the FP64 finest level at a region's nodes, for the mixed
// form's correction equation A e = r: r = b - A x formed in FP64 by the
// same products in the same order as the residual kernel, rounded to FP32.
// The region's x (FP64) is first staged in the LDS rows themselves (a row's
// x and b arrays, two FP32 rows, hold one FP64 row); once every wave has
// formed its rows' r in registers, each row gets x = 0 (the correction
// starts from zero) and b = r.  At the output nodes r also goes into F.b
// (for the passes after this one) and r^2 into the workgroup's partial sum
// of the norm.  A wave holds region rows wave, wave + NWAVE, ... : at most
// RESID_ROWS of them, so R <= RESID_ROWS * NWAVE.  Returns false when the
// workgroup stops here (solve finished, or only the residual was asked).
constexpr int RESID_ROWS = 12;
template <typename T, int K, bool B1, int NCOL, int P>
__device__ bool wresid(const Level<T>& F, const Level<double>& X, const WMap& m, MG_LDS T* lds, MG_LDS double* xs,
                       int R, int TX, int TY, bool only, double* sh) {
  constexpr int PD = P / 2;  // FP64 values per LDS row
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int la = lane, lb = lane + 64;
  const bool oka = m.col_ok(la), okb = m.col_ok(lb);
  const int ga = m.gi(la), gb = m.gi(lb);
  // r is needed at the unknowns inside the region's outer ring
  const bool na = oka && la >= 1, nb = okb && lb <= WW - 2;
  const int done = F.st->done;
  double ba[RESID_ROWS], bb[RESID_ROWS];
#pragma unroll
  for (int u = 0; u < RESID_ROWS; ++u) {
    const int lj = wave + u * NWAVE;
    ba[u] = bb[u] = 0.0;
    if (lj >= 1 && lj <= R - 2 && m.row_ok(lj)) {
      const double* row = X.b + (size_t)m.wrapj(m.gj(lj)) * X.pitch;
      if (na) ba[u] = row[ga];
      if (nb) bb[u] = row[gb];
    }
  }
  // x of the region, Dirichlet boundary nodes (and nodes off the grid) as 0
  for (int lj0 = wave; lj0 < R; lj0 += NWAVE * ULR) {
    double xa[ULR], xb[ULR];
#pragma unroll
    for (int u = 0; u < ULR; ++u) {
      const int lj = lj0 + u * NWAVE;
      xa[u] = xb[u] = 0.0;
      if (lj < R && m.row_ok(lj)) {
        const double* row = X.x + (size_t)m.wrapj(m.gj(lj)) * X.pitch;
        if (oka) xa[u] = row[ga];
        if (okb) xb[u] = row[gb];
      }
    }
#pragma unroll
    for (int u = 0; u < ULR; ++u) {
      const int lj = lj0 + u * NWAVE;
      if (lj >= R) break;
      xs[lj * PD + la] = xa[u];
      xs[lj * PD + lb] = xb[u];
    }
  }
  __syncthreads();
  if (done) return false;

  Cf<double> cola{}, colb{};
  if constexpr (K == ST9 && B1) {
    cola = coefs<K>(X, na ? ga : 1, 0, 0);
    colb = coefs<K>(X, nb ? gb : 1, 0, 0);
  }
  const bool oa = la >= m.H && la < m.H + TX, ob = lb < m.H + TX;  // output columns
  float ra[RESID_ROWS], rb[RESID_ROWS];
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < RESID_ROWS; ++u) {
    const int lj = wave + u * NWAVE;
    ra[u] = rb[u] = 0.f;
    if (!(lj >= 1 && lj <= R - 2 && m.row_ok(lj))) continue;
    const int gj = m.wrapj(m.gj(lj));
    const bool orow = lj >= m.Hy && lj < m.Hy + TY && m.gj(lj) < F.ny;
    auto defect = [&](int li, int gi, const Cf<double>& col, double bp) {
      const MG_LDS double* p = xs + (lj - 1) * PD + li;
      Nbr<double> v;
      v.sw = p[-1];
      v.s = p[0];
      v.se = p[1];
      v.w = p[PD - 1];
      v.c = p[PD];
      v.e = p[PD + 1];
      v.nw = p[2 * PD - 1];
      v.n = p[2 * PD];
      v.ne = p[2 * PD + 1];
      const Cf<double> a = (K == ST9 && !B1) ? coefs<K>(X, gi, gj, wrap_dn(gj, X.ny, X.py)) : col;
      return defect_v<K>(X, a, v, bp);
    };
    if (na) {
      const double d = defect(la, ga, cola, ba[u]);
      ra[u] = (float)d;
      if (orow && oa) {
        F.b[(size_t)gj * F.pitch + ga] = ra[u];
        acc += d * d;
      }
    }
    if (nb) {
      const double d = defect(lb, gb, colb, bb[u]);
      rb[u] = (float)d;
      if (orow && ob) {
        F.b[(size_t)gj * F.pitch + gb] = rb[u];
        acc += d * d;
      }
    }
  }
  const double part = wg_sum(acc, sh);  // ends with a barrier: the staged x is no longer read
  if (threadIdx.x == 0) X.st->partial[blockIdx.x] = part;
  if (only) return false;
  const int ca = wcol(la), cb = wcol(lb);
#pragma unroll
  for (int u = 0; u < RESID_ROWS; ++u) {
    const int lj = wave + u * NWAVE;
    if (lj >= R) break;
    MG_LDS T* r = lds + lj * P;
    r[ca] = (T)0;
    r[cb] = (T)0;
    r[WW + ca] = (T)ra[u];
    r[WW + cb] = (T)rb[u];
    if constexpr (NCOL == 0) {
      r[2 * WW + ca] = (T)0;
      r[2 * WW + cb] = (T)0;
    }
  }
  return true;
}

template <typename T, int K, bool FINE, int NCOL, bool B1>
__global__ void __launch_bounds__(FT) k_pre_w(const Level<T>* __restrict__ Fs, const Level<T>* __restrict__ Cs,
                                              int TY, int H, int Hy, int ntx, int nty, int nsteps, T omega,
                                              int start, const Level<double>* __restrict__ X64s) {
  constexpr int P = wide_narr<NCOL>() * WW;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Level<T> F = Fs[blockIdx.z];
  if (batched_done(F.st)) return;
  const Level<T> C = Cs[blockIdx.z];
  int tx, ty;
  tile_coords(ntx, nty, tx, ty);
  const int TX = WW - 2 * H, R = TY + 2 * Hy;
  MG_LDS T* lds = lds_cast<T>(smem_raw);
  MG_LDS T* bl = lds + R * P;
  const WMap m{tx * TX, ty * TY, H, Hy, F.nx, F.ny, F.py};
  const int wave = wave_id(), lane = threadIdx.x & 63;
  WBands<T> bands{};
  if constexpr (B1) bands = wfetch_bands(F, m);

  // (only the FP32 finest level of the mixed form forms its residual, not
  // with per-node 9-point coefficients, whose loads would cost the pass its
  // occupancy)
  constexpr bool MIX = FINE && std::is_same<T, float>::value && (K != ST9 || B1);
  if (MIX && start >= PRE_RESID) {
    if constexpr (MIX) {
      __shared__ double sh[FT / 64];
      if (!wresid<T, K, B1, NCOL, P>(F, X64s[blockIdx.z], m, lds, lds_cast<double>(smem_raw), R, TX, TY,
                                     start == PRE_RESID_ONLY, sh))
        return;
    }
  } else {
    const int la = lane, lb = lane + 64;
    const int ca = wcol(la), cb = wcol(lb);
    const bool oka = m.col_ok(la), okb = m.col_ok(lb);
    const int ga = m.gi(la), gb = m.gi(lb);
    for (int lj0 = wave; lj0 < R; lj0 += NWAVE * ULR) {
      T xa[ULR], xb[ULR], ba[ULR], bb[ULR];
#pragma unroll
      for (int u = 0; u < ULR; ++u) {
        const int lj = lj0 + u * NWAVE;
        xa[u] = xb[u] = ba[u] = bb[u] = (T)0;
        if (lj < R && m.row_ok(lj)) {
          const size_t row = (size_t)m.wrapj(m.gj(lj)) * F.pitch;
          if (oka) {
            if (!start) xa[u] = F.x[row + ga];
            ba[u] = F.b[row + ga];
          }
          if (okb) {
            if (!start) xb[u] = F.x[row + gb];
            bb[u] = F.b[row + gb];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < ULR; ++u) {
        const int lj = lj0 + u * NWAVE;
        if (lj >= R) break;
        MG_LDS T* r = lds + lj * P;
        r[ca] = xa[u];
        r[cb] = xb[u];
        r[WW + ca] = ba[u];
        r[WW + cb] = bb[u];
        if constexpr (NCOL == 0) {
          r[2 * WW + ca] = (T)0;
          r[2 * WW + cb] = (T)0;
        }
      }
    }
  }
  if constexpr (B1) wstore_bands(bl, bands);
  const int done = F.st->done;
  __syncthreads();
  if (done) return;

  const int xsrc = wsmooth<T, K, NCOL, B1>(F, m, lds, bl, R, nsteps, omega);
  if (xsrc == 0)
    wsweep_region<T, K, NCOL, B1, 0, 1>(F, m, lds, bl, R, H - 1, Hy - 1, omega);
  else
    wsweep_region<T, K, NCOL, B1, 2, 1>(F, m, lds, bl, R, H - 1, Hy - 1, omega);
  __syncthreads();

  // full weighting at the coarse nodes of the tile; zero coarse start
  {
    const int ca = TX >> 1, nrb = TY >> 1;
    const int li = H + 2 * lane, A = li >> 1;
    const int I = (m.i0 >> 1) + lane;
    const bool iok = lane < ca && I >= 1 && I <= C.nx - 2;
    const int lo = C.py ? 0 : 1, hi = C.py ? C.ny - 1 : C.ny - 2;
    for (int rb = wave; rb < nrb; rb += NWAVE) {
      const int J = (m.j0 >> 1) + rb;
      if (!iok || J < lo || J > hi) continue;
      const MG_LDS T* p = lds + WW + (Hy + 2 * rb - 1) * P + A;
      const Nbr<T> d = (H & 1) ? wgather<T, ST9, P, 1, true>(p) : wgather<T, ST9, P, 0, true>(p);
      const T g = fw_combine(fw_row(d.sw, d.s, d.se), fw_row(d.w, d.c, d.e), fw_row(d.nw, d.n, d.ne));
      const size_t q = (size_t)J * C.pitch + I;
      C.b[q] = g;
      C.x[q] = (T)0;
    }
  }
  // smoothed iterate of the output nodes -> ping-pong buffer
  {
    const int la = H + lane, lb = H + lane + 64;
    const bool oka = m.col_ok(la), okb = lb < H + TX && m.col_ok(lb);
    const int ga = m.gi(la), gb = m.gi(lb);
    for (int lj = Hy + wave; lj < Hy + TY; lj += NWAVE) {
      const int gj = m.gj(lj);
      if (!m.row_ok(lj) || gj >= F.ny) continue;
      const MG_LDS T* r = lds + lj * P + xsrc * WW;
      T* row = F.t + (size_t)gj * F.pitch;
      if (oka) row[ga] = r[wcol(la)];
      if (okb) row[gb] = r[wcol(lb)];
    }
  }
}

// Residual norm contribution of the output nodes of column parity Q.
template <typename T, int K, bool B1, int P, int Q>
__device__ double wnorm_part(const Level<T>& F, const WMap& m, const MG_LDS T* lds, const MG_LDS T* bl, int xsrc,
                             int TX, int TY) {
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int H = m.H;
  const int li = H + ((H ^ Q) & 1) + 2 * lane;
  if (!(li < H + TX && m.col_ok(li))) return 0.0;
  const int A = li >> 1, gi = m.gi(li);
  Cf<T> col{};
  if constexpr (K == ST9 && B1) col = wcoef_cols<T, Q>(bl, A);
  constexpr int own = Q ? WH : 0;
  double acc = 0.0;
  for (int lj = m.Hy + wave; lj < m.Hy + TY; lj += NWAVE) {
    if (!m.row_ok(lj) || m.gj(lj) >= F.ny) continue;
    const Nbr<T> v = wgather<T, K, P, Q, true>(lds + xsrc * WW + (lj - 1) * P + A);
    const T d = defect_v<K>(F, wcoef<T, K, B1>(F, m, col, gi, lj), v, lds[lj * P + WW + own + A]);
    acc += (double)d * (double)d;
  }
  return acc;
}

template <typename T, int K, bool FINE, int NCOL, bool B1>
__global__ void __launch_bounds__(FT) k_post_w(const Level<T>* __restrict__ Fs, const Level<T>* __restrict__ Cs,
                                               int TY, int H, int Hy, int ntx, int nty, int nsteps, T omega,
                                               int mode, const Level<double>* __restrict__ X64s) {
  constexpr int P = wide_narr<NCOL>() * WW;
  constexpr int CW = WH + 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double sh[FT / 64];
  const Level<T> F = Fs[blockIdx.z];
  SolveState* st = F.st;
  if (batched_done(st)) return;
  const Level<T> C = Cs[blockIdx.z];
  const bool wtd = F.wl != nullptr;  // adaptive omega_l
  const T wv = wtd ? *F.wl : (T)1;
  int tx, ty;
  tile_coords(ntx, nty, tx, ty);
  const int TX = WW - 2 * H, R = TY + 2 * Hy;
  const int CR = (R >> 1) + 2;
  MG_LDS T* lds = lds_cast<T>(smem_raw);
  MG_LDS T* ec = lds + R * P;
  MG_LDS T* bl = ec + CW * CR;
  const WMap m{tx * TX, ty * TY, H, Hy, F.nx, F.ny, F.py};
  const int wave = wave_id(), lane = threadIdx.x & 63;
  WBands<T> bands{};
  if constexpr (B1) bands = wfetch_bands(F, m);

  // Every global load of the region's first rows, of the coarse correction
  // and (POST_MIXED) of the FP64 iterate at the wave's first output rows is
  // issued before the first wait, so the pass waits on memory about once.
  const int la = lane, lb = lane + 64;
  const int ca = wcol(la), cb = wcol(lb);
  const bool oka = m.col_ok(la), okb = m.col_ok(lb);
  const int ga = m.gi(la), gb = m.gi(lb);
  T ta[ULR], tb[ULR], ba[ULR], bb[ULR];
  auto load_rows = [&](int lj0, auto nrows) {
    constexpr int NR = decltype(nrows)::value;
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int lj = lj0 + u * NWAVE;
      ta[u] = tb[u] = ba[u] = bb[u] = (T)0;
      if (lj < R && m.row_ok(lj)) {
        const size_t row = (size_t)m.wrapj(m.gj(lj)) * F.pitch;
        if (oka) {
          ta[u] = F.t[row + ga];
          ba[u] = F.b[row + ga];
        }
        if (okb) {
          tb[u] = F.t[row + gb];
          bb[u] = F.b[row + gb];
        }
      }
    }
  };
  load_rows(wave, std::integral_constant<int, ULR>{});

  const int oa = H + lane, ob = H + lane + 64;
  const bool ooka = m.col_ok(oa), ookb = ob < H + TX && m.col_ok(ob);
  const int oga = m.gi(oa), ogb = m.gi(ob);
  // (only the FP32 finest level runs POST_MIXED)
  constexpr bool MIX = FINE && std::is_same<T, float>::value;
  const bool mixed = mode == POST_MIXED || mode == POST_MIXED_KEEP;
  double pxa[UL], pxb[UL];
  if (MIX && mixed) {
    const Level<double>& X = X64s[blockIdx.z];
#pragma unroll
    for (int u = 0; u < UL; ++u) {
      const int lj = Hy + wave + u * NWAVE, gj = m.gj(lj);
      pxa[u] = pxb[u] = 0.0;
      if (lj < Hy + TY && m.row_ok(lj) && gj < F.ny) {
        const double* xrow = X.x + (size_t)gj * X.pitch;
        if (ooka) pxa[u] = xrow[oga];
        if (ookb) pxb[u] = xrow[ogb];
      }
    }
  }

  // coarse correction covering the region
  const int cI0 = m.gi(0) >> 1, cJ0 = m.gj(0) >> 1;
  {
    const int clo = C.py ? 0 : 1, chi = C.py ? C.ny - 1 : C.ny - 2;
    const int Ia = cI0 + lane, Ib = cI0 + lane + 64;
    const bool eoka = Ia >= 1 && Ia <= C.nx - 2, eokb = lane + 64 < CW && Ib >= 1 && Ib <= C.nx - 2;
    for (int r0 = wave; r0 < CR; r0 += NWAVE * UL) {
      T va[UL], vb[UL];
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        int J = cJ0 + r0 + u * NWAVE;
        if (C.py) {
          while (J < 0) J += C.ny;
          while (J >= C.ny) J -= C.ny;
        }
        va[u] = vb[u] = (T)0;
        if (r0 + u * NWAVE < CR && J >= clo && J <= chi) {
          const T* row = C.x + (size_t)J * C.pitch;
          if (eoka) va[u] = row[Ia];
          if (eokb) vb[u] = row[Ib];
        }
      }
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int r = r0 + u * NWAVE;
        if (r >= CR) break;
        ec[r * CW + lane] = va[u];
        if (lane + 64 < CW) ec[r * CW + lane + 64] = vb[u];
      }
    }
  }
  if constexpr (B1) wstore_bands(bl, bands);
  __syncthreads();
  {
    const int ea = (ga >> 1) - cI0, eb = (gb >> 1) - cI0;
    auto store_rows = [&](int lj0, auto nrows) {
      constexpr int NR = decltype(nrows)::value;
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int lj = lj0 + u * NWAVE;
        if (lj >= R) break;
        const int gj = m.gj(lj);
        T xa = (T)0, xb = (T)0;
        if (m.row_ok(lj)) {
          const MG_LDS T* e0 = ec + ((gj >> 1) - cJ0) * CW;
          const MG_LDS T* e1 = e0 + CW;
          const int oy = gj & 1;
          if (oka) xa = add_correction(ta[u], prolong_combine(e0[ea], e0[ea + 1], e1[ea], e1[ea + 1], ga & 1, oy), wtd, wv);
          if (okb) xb = add_correction(tb[u], prolong_combine(e0[eb], e0[eb + 1], e1[eb], e1[eb + 1], gb & 1, oy), wtd, wv);
        }
        MG_LDS T* r = lds + lj * P;
        r[ca] = xa;
        r[cb] = xb;
        r[WW + ca] = ba[u];
        r[WW + cb] = bb[u];
        if constexpr (NCOL == 0) {
          r[2 * WW + ca] = (T)0;
          r[2 * WW + cb] = (T)0;
        }
      }
    };
    store_rows(wave, std::integral_constant<int, ULR>{});
    for (int lj0 = wave + NWAVE * ULR; lj0 < R; lj0 += NWAVE * UL) {
      load_rows(lj0, std::integral_constant<int, UL>{});
      store_rows(lj0, std::integral_constant<int, UL>{});
    }
  }
  const int done = F.st->done;
  __syncthreads();
  if (done) return;

  const int xsrc = wsmooth<T, K, NCOL, B1>(F, m, lds, bl, R, nsteps, omega);

  if (MIX && mixed) {
    const Level<double>& X = X64s[blockIdx.z];
    const bool zero_e = mode == POST_MIXED;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->pending = 1;
    for (int lj0 = Hy + wave; lj0 < Hy + TY; lj0 += NWAVE * UL) {
      double xa[UL], xb[UL];
      const bool first = lj0 == Hy + wave;  // loaded before the sweeps
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int lj = lj0 + u * NWAVE, gj = m.gj(lj);
        xa[u] = pxa[u];
        xb[u] = pxb[u];
        if (!first) {
          xa[u] = xb[u] = 0.0;
          if (lj < Hy + TY && m.row_ok(lj) && gj < F.ny) {
            const double* xrow = X.x + (size_t)gj * X.pitch;
            if (ooka) xa[u] = xrow[oga];
            if (ookb) xb[u] = xrow[ogb];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int lj = lj0 + u * NWAVE, gj = m.gj(lj);
        if (!(lj < Hy + TY && m.row_ok(lj) && gj < F.ny)) continue;
        const MG_LDS T* r = lds + lj * P + xsrc * WW;
        double* xrow = X.x + (size_t)gj * X.pitch;
        T* row = F.x + (size_t)gj * F.pitch;
        if (ooka) {
          xrow[oga] = xa[u] + (double)r[wcol(oa)];
          if (zero_e) row[oga] = (T)0;
        }
        if (ookb) {
          xrow[ogb] = xb[u] + (double)r[wcol(ob)];
          if (zero_e) row[ogb] = (T)0;
        }
      }
    }
  } else {
    for (int lj = Hy + wave; lj < Hy + TY; lj += NWAVE) {
      const int gj = m.gj(lj);
      if (!m.row_ok(lj) || gj >= F.ny) continue;
      const MG_LDS T* r = lds + lj * P + xsrc * WW;
      T* row = F.x + (size_t)gj * F.pitch;
      if (ooka) row[oga] = r[wcol(oa)];
      if (ookb) row[ogb] = r[wcol(ob)];
    }
  }
  if (mode == POST_NORM) {
    double acc = wnorm_part<T, K, B1, P, 0>(F, m, lds, bl, xsrc, TX, TY);
    acc += wnorm_part<T, K, B1, P, 1>(F, m, lds, bl, xsrc, TX, TY);
    const double part = wg_sum(acc, sh);
    if (threadIdx.x == 0) st->partial[blockIdx.x] = part;
  }
}

// ------------------------------------------------------------------ launchers

TileGeom tile_geom(int nx, int ny, int TX, int TY, int H) {
  TileGeom g;
  g.TX = TX;
  g.TY = TY;
  g.H = H;
  g.Hy = H;
  g.ntx = (nx + TX - 1) / TX;
  g.nty = (ny + TY - 1) / TY;
  g.wide = 0;
  return g;
}

TileGeom wide_geom(int nx, int ny, int TY, int H, int Hy) {
  TileGeom g = tile_geom(nx, ny, WW - 2 * H, TY, H);
  g.Hy = Hy;
  g.wide = 1;
  return g;
}

int wide_width() { return WW; }

template <typename T>
size_t pre_lds_bytes(const TileGeom& g, int ncol) {
  const size_t narr = ncol == 0 ? 3 : 2;
  if (g.wide) return ((g.TY + 2 * g.Hy) * narr * WW + NBANDS * WW) * sizeof(T);
  const size_t W = g.TX + 2 * g.H, R = g.TY + 2 * g.H;
  return (W * R * narr + NBANDS * W) * sizeof(T);
}

template <typename T>
size_t post_lds_bytes(const TileGeom& g, int ncol) {
  const size_t narr = ncol == 0 ? 3 : 2;
  if (g.wide) {
    const size_t R = g.TY + 2 * g.Hy;
    return (R * narr * WW + (WH + 2) * ((R >> 1) + 2) + NBANDS * WW) * sizeof(T);
  }
  const size_t W = g.TX + 2 * g.H, R = g.TY + 2 * g.H;
  const size_t CW = (W >> 1) + 2, CR = (R >> 1) + 2;
  return (W * R * narr + CW * CR + NBANDS * W) * sizeof(T);
}

// Kernel variants by stencil, finest level, smoother (Jacobi, red-black,
// four-colour), 1-D bands and tile shape.  Red-black is not defined for
// 9-point operators and 1-D bands only exist for them: those variants are
// nullptr.
template <typename T>
using PreFn = void (*)(const Level<T>*, const Level<T>*, int, int, int, int, int, int, T);
template <typename T>
using PostFn = void (*)(const Level<T>*, const Level<T>*, int, int, int, int, int, int, T, int, const Level<double>*);
template <typename T>
using PreWFn = void (*)(const Level<T>*, const Level<T>*, int, int, int, int, int, int, T, int,
                        const Level<double>*);
template <typename T>
using PostWFn = void (*)(const Level<T>*, const Level<T>*, int, int, int, int, int, int, T, int,
                         const Level<double>*);

// f(NCOL, B1) -> kernel for the valid (stencil, smoother, bands) triples.
#define MG_VARIANT(K, ncol, b1, F)                                                        \
  do {                                                                                    \
    if constexpr (K == ST5) {                                                             \
      if (b1) return nullptr;                                                             \
      if (ncol == 0) return F(0, false);                                                  \
      if (ncol == 2) return F(2, false);                                                  \
      if (ncol == 4) return F(4, false);                                                  \
    } else {                                                                              \
      if (ncol == 0) return b1 ? F(0, true) : F(0, false);                                \
      if (ncol == 4) return b1 ? F(4, true) : F(4, false);                                \
    }                                                                                     \
    return nullptr;                                                                       \
  } while (0)

template <typename T, int K, bool FINE>
PreFn<T> pre_fn(int ncol, bool b1) {
#define MG_F(NC, B) k_pre<T, K, FINE, NC, B>
  MG_VARIANT(K, ncol, b1, MG_F);
#undef MG_F
}

template <typename T, int K, bool FINE>
PostFn<T> post_fn(int ncol, bool b1) {
#define MG_F(NC, B) k_post<T, K, FINE, NC, B>
  MG_VARIANT(K, ncol, b1, MG_F);
#undef MG_F
}

template <typename T, int K, bool FINE>
PreWFn<T> pre_w_fn(int ncol, bool b1) {
#define MG_F(NC, B) k_pre_w<T, K, FINE, NC, B>
  MG_VARIANT(K, ncol, b1, MG_F);
#undef MG_F
}

template <typename T, int K, bool FINE>
PostWFn<T> post_w_fn(int ncol, bool b1) {
#define MG_F(NC, B) k_post_w<T, K, FINE, NC, B>
  MG_VARIANT(K, ncol, b1, MG_F);
#undef MG_F
}

#undef MG_VARIANT

template <typename T>
PreFn<T> pick_pre(int kind, bool oned, bool fine, int ncol) {
  if (kind == ST5) return fine ? pre_fn<T, ST5, true>(ncol, false) : pre_fn<T, ST5, false>(ncol, false);
  return fine ? pre_fn<T, ST9, true>(ncol, oned) : pre_fn<T, ST9, false>(ncol, oned);
}

template <typename T>
PostFn<T> pick_post(int kind, bool oned, bool fine, int ncol) {
  if (kind == ST5) return fine ? post_fn<T, ST5, true>(ncol, false) : post_fn<T, ST5, false>(ncol, false);
  return fine ? post_fn<T, ST9, true>(ncol, oned) : post_fn<T, ST9, false>(ncol, oned);
}

template <typename T>
PreWFn<T> pick_pre_w(int kind, bool oned, bool fine, int ncol) {
  if (kind == ST5) return fine ? pre_w_fn<T, ST5, true>(ncol, false) : pre_w_fn<T, ST5, false>(ncol, false);
  return fine ? pre_w_fn<T, ST9, true>(ncol, oned) : pre_w_fn<T, ST9, false>(ncol, oned);
}

template <typename T>
PostWFn<T> pick_post_w(int kind, bool oned, bool fine, int ncol) {
  if (kind == ST5) return fine ? post_w_fn<T, ST5, true>(ncol, false) : post_w_fn<T, ST5, false>(ncol, false);
  return fine ? post_w_fn<T, ST9, true>(ncol, oned) : post_w_fn<T, ST9, false>(ncol, oned);
}

template <typename T>
hipError_t prepare_fused() {
  for (int kind : {(int)ST5, (int)ST9})
    for (int oned = 0; oned < 2; ++oned)
      for (int fine = 0; fine < 2; ++fine)
        for (int ncol : {0, 2, 4}) {
          const void* ks[4] = {(const void*)pick_pre<T>(kind, oned, fine, ncol),
                               (const void*)pick_post<T>(kind, oned, fine, ncol),
                               (const void*)pick_pre_w<T>(kind, oned, fine, ncol),
                               (const void*)pick_post_w<T>(kind, oned, fine, ncol)};
          for (const void* k : ks) {
            if (!k) continue;
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)FUSED_LDS_MAX);
            if (e != hipSuccess) return e;
          }
        }
  return hipSuccess;
}

bool pre_resid_fits(const TileGeom& g) { return g.wide && g.TY + 2 * g.Hy <= RESID_ROWS * NWAVE; }
bool pre_resid_kind(int kind, bool oned) { return kind == ST5 || oned; }

template <typename T>
hipError_t launch_pre(const Level<T>* Fs, const Level<T>* Cs, const TileGeom& g, int nsteps, int ncol, T omega,
                      int kind, bool oned, bool fine, int nslots, hipStream_t st, int mode,
                      const Level<double>* X64s) {
  const dim3 grid(g.ntx * g.nty, 1, nslots);
  const size_t lds = pre_lds_bytes<T>(g, ncol);
  if (mode < PRE_LOAD || mode > PRE_RESID_ONLY) return hipErrorInvalidValue;
  // residual modes: FP32 finest level, wide tiles
  if (mode >= PRE_RESID &&
      !(std::is_same<T, float>::value && fine && X64s && pre_resid_fits(g) && pre_resid_kind(kind, oned)))
    return hipErrorInvalidValue;
  if (g.wide) {
    PreWFn<T> k = pick_pre_w<T>(kind, oned, fine, ncol);
    if (!k || g.TX != WW - 2 * g.H) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, grid, dim3(FT), lds, st, Fs, Cs, g.TY, g.H, g.Hy, g.ntx, g.nty, nsteps, omega, mode, X64s);
  } else {
    PreFn<T> k = pick_pre<T>(kind, oned, fine, ncol);
    if (!k || mode != PRE_LOAD) return hipErrorInvalidValue;  // zero start: wide tiles only
    hipLaunchKernelGGL(k, grid, dim3(FT), lds, st, Fs, Cs, g.TX, g.TY, g.H, g.ntx, g.nty, nsteps, omega);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_post(const Level<T>* Fs, const Level<T>* Cs, const TileGeom& g, int nsteps, int ncol, T omega,
                       int mode, const Level<double>* X64s, int kind, bool oned, bool fine, int nslots,
                       hipStream_t st, bool with_finish) {
  const dim3 grid(g.ntx * g.nty, 1, nslots);
  const size_t lds = post_lds_bytes<T>(g, ncol);
  if (g.wide) {
    PostWFn<T> k = pick_post_w<T>(kind, oned, fine, ncol);
    if (!k || g.TX != WW - 2 * g.H) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, grid, dim3(FT), lds, st, Fs, Cs, g.TY, g.H, g.Hy, g.ntx, g.nty, nsteps, omega, mode, X64s);
  } else {
    PostFn<T> k = pick_post<T>(kind, oned, fine, ncol);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, grid, dim3(FT), lds, st, Fs, Cs, g.TX, g.TY, g.H, g.ntx, g.nty, nsteps, omega, mode,
                       X64s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || mode != POST_NORM || !with_finish) return e;
  return launch_norm_finish<T>(Fs, g.ntx * g.nty, NORM_CHECK, nslots, st);
}

#define MG_FUSED_INSTANTIATE(T)                                                                                    \
  template size_t pre_lds_bytes<T>(const TileGeom&, int);                                                          \
  template size_t post_lds_bytes<T>(const TileGeom&, int);                                                         \
  template hipError_t prepare_fused<T>();                                                                          \
  template hipError_t launch_pre<T>(const Level<T>*, const Level<T>*, const TileGeom&, int, int, T, int, bool,     \
                                    bool, int, hipStream_t, int, const Level<double>*);                            \
  template hipError_t launch_post<T>(const Level<T>*, const Level<T>*, const TileGeom&, int, int, T, int,         \
                                     const Level<double>*, int, bool, bool, int, hipStream_t, bool);

MG_FUSED_INSTANTIATE(double)
MG_FUSED_INSTANTIATE(float)

}  // namespace mg
