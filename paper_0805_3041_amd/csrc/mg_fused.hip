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
#include "mg_fused.h"

namespace mg {

constexpr int FT = 512;  // threads per tile workgroup

struct TileMap {
  int i0, j0, H, nx, ny, py;
  __device__ __forceinline__ int gi(int li) const { return i0 - H + li; }
  __device__ __forceinline__ int gj(int lj) const { return j0 - H + lj; }  // not wrapped
  __device__ __forceinline__ int wrapj(int j) const { return py ? ((j % ny) + ny) % ny : j; }
  __device__ __forceinline__ bool unknown(int i, int j) const {
    if (i < 1 || i > nx - 2) return false;
    return py ? true : (j >= 1 && j <= ny - 2);
  }
};

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

// One Gauss-Seidel colour sweep over the region shrunk by s.
template <typename T, int K>
__device__ void tile_colour(const Level<T>& L, const TileMap& m, MG_LDS T* x, const MG_LDS T* b, int W, int R, int s,
                            int c, int ncol) {
  constexpr int NB = nbatch(K);
  const int lo = s, hiW = W - s, hiR = R - s;
  int nk, nr, lj0, rstep, li0 = 0;
  if (ncol == 2) {
    nk = (hiW - lo + 1) >> 1;
    nr = hiR - lo;
    lj0 = lo;
    rstep = 1;
  } else {
    lj0 = lo + (((m.gj(lo) & 1) != (c >> 1)) ? 1 : 0);
    li0 = lo + (((m.gi(lo) & 1) != (c & 1)) ? 1 : 0);
    nr = lj0 < hiR ? (hiR - lj0 + 1) >> 1 : 0;
    nk = li0 < hiW ? (hiW - li0 + 1) >> 1 : 0;
    rstep = 2;
  }
  const int n = nr * nk;
  if (n <= 0) return;
  const FDiv dk(nk);
  for (int base = threadIdx.x; base < n; base += FT * NB) {
    int pos[NB], gi[NB], gjw[NB];
    bool ok[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = base + u * FT;
      ok[u] = false;
      pos[u] = gi[u] = gjw[u] = 0;
      if (idx < n) {
        const int r = dk.q(idx);
        const int k = idx - r * nk;
        const int lj = lj0 + rstep * r;
        const int gj = m.gj(lj);
        const int li = ncol == 2 ? lo + 2 * k + ((((m.gi(lo) + gj) & 1) != c) ? 1 : 0) : li0 + 2 * k;
        const int g = m.gi(li);
        if (li < hiW && m.unknown(g, gj)) {
          ok[u] = true;
          pos[u] = lj * W + li;
          gi[u] = g;
          gjw[u] = m.wrapj(gj);
        }
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
      a[u] = coefs<K>(L, gi[u], gjw[u], wrap_dn(gjw[u], L.ny, L.py));
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (ok[u]) x[pos[u]] = gs_v<K>(L, a[u], v[u], bp[u]);
  }
}

// Region nodes (shrunk by s) that are unknowns, NB per thread per round:
// f(pos, gi, gj_wrapped) is called for the loads, g(...) for the stores.
template <typename T, int K>
__device__ void tile_jacobi(const Level<T>& L, const TileMap& m, const MG_LDS T* src, MG_LDS T* dst,
                            const MG_LDS T* b, int W, int R, int s, T omega) {
  constexpr int NB = nbatch(K);
  const int cols = W - 2 * s, n = (R - 2 * s) * cols;
  const FDiv dc(cols);
  for (int base = threadIdx.x; base < n; base += FT * NB) {
    int pos[NB], gi[NB], gjw[NB];
    bool ok[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = base + u * FT;
      ok[u] = false;
      pos[u] = gi[u] = gjw[u] = 0;
      if (idx < n) {
        const int r = dc.q(idx);
        const int lj = s + r, li = s + idx - r * cols;
        const int gj = m.gj(lj), g = m.gi(li);
        if (m.unknown(g, gj)) {
          ok[u] = true;
          pos[u] = lj * W + li;
          gi[u] = g;
          gjw[u] = m.wrapj(gj);
        }
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
      a[u] = coefs<K>(L, gi[u], gjw[u], wrap_dn(gjw[u], L.ny, L.py));
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (ok[u]) dst[pos[u]] = jac_v<K>(L, a[u], v[u], bp[u], omega);
  }
}

// Defect b - A x on the region shrunk by s, written in place into b (a
// node's defect reads only its own b); 0 at non-unknowns.
template <typename T, int K>
__device__ void tile_defect(const Level<T>& L, const TileMap& m, const MG_LDS T* x, MG_LDS T* b, int W, int R,
                            int s) {
  constexpr int NB = nbatch(K);
  const int cols = W - 2 * s, n = (R - 2 * s) * cols;
  const FDiv dc(cols);
  for (int base = threadIdx.x; base < n; base += FT * NB) {
    int pos[NB], gi[NB], gjw[NB];
    bool ok[NB], in[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = base + u * FT;
      ok[u] = in[u] = false;
      pos[u] = gi[u] = gjw[u] = 0;
      if (idx < n) {
        in[u] = true;
        const int r = dc.q(idx);
        const int lj = s + r, li = s + idx - r * cols;
        const int gj = m.gj(lj), g = m.gi(li);
        pos[u] = lj * W + li;
        if (m.unknown(g, gj)) {
          ok[u] = true;
          gi[u] = g;
          gjw[u] = m.wrapj(gj);
        }
      }
    }
    Nbr<T> v[NB];
    Cf<T> a[NB];
    T bp[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (!ok[u]) continue;
      v[u] = gather<K>(L, LXW<T>{x + pos[u], W}, true);
      bp[u] = b[pos[u]];
      a[u] = coefs<K>(L, gi[u], gjw[u], wrap_dn(gjw[u], L.ny, L.py));
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (in[u]) b[pos[u]] = ok[u] ? defect_v<K>(L, a[u], v[u], bp[u]) : (T)0;
  }
}

// nsteps smoothing steps on the region; returns the LDS array holding the
// result (x, or t after an odd number of Jacobi steps).
template <typename T, int K>
__device__ MG_LDS T* tile_smooth(const Level<T>& L, const TileMap& m, MG_LDS T* x, MG_LDS T* t, const MG_LDS T* b,
                                 int W, int R, int nsteps, int ncol, T omega) {
  int s = 1;
  if (ncol == 0) {
    MG_LDS T* src = x;
    MG_LDS T* dst = t;
    for (int k = 0; k < nsteps; ++k, ++s) {
      tile_jacobi<T, K>(L, m, src, dst, b, W, R, s, omega);
      __syncthreads();
      MG_LDS T* tmp = src;
      src = dst;
      dst = tmp;
    }
    return src;
  }
  for (int k = 0; k < nsteps; ++k) {
    for (int c = 0; c < ncol; ++c, ++s) {
      tile_colour<T, K>(L, m, x, b, W, R, s, c, ncol);
      __syncthreads();
    }
  }
  return x;
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

// ------------------------------------------------------------------ pre-pass

// FINE: instantiation used on the finest level only (a separate symbol, so
// profiles and timings of the finest pass are not mixed with coarser ones).
template <typename T, int K, bool FINE>
__global__ void __launch_bounds__(FT) k_pre(const Level<T>* __restrict__ Fs, const Level<T>* __restrict__ Cs, int TX,
                                            int TY, int H, int ntx, int nty, int nsteps, int ncol, T omega) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Level<T> F = Fs[blockIdx.z];
  if (F.st->done) return;
  const Level<T> C = Cs[blockIdx.z];
  int tx, ty;
  tile_coords(ntx, nty, tx, ty);
  const int W = TX + 2 * H, R = TY + 2 * H;
  MG_LDS T* x = lds_cast<T>(smem_raw);
  MG_LDS T* b = x + W * R;
  MG_LDS T* t = b + W * R;  // Jacobi only
  const TileMap m{tx * TX, ty * TY, H, F.nx, F.ny, F.py};

  const FDiv dW(W);
  for (int idx = threadIdx.x; idx < W * R; idx += FT) {
    const int lj = dW.q(idx), li = idx - lj * W;
    const int gi = m.gi(li), gj = m.gj(lj);
    T xv = (T)0, bv = (T)0;
    if (m.unknown(gi, gj)) {
      const size_t p = (size_t)m.wrapj(gj) * F.pitch + gi;
      xv = F.x[p];
      bv = F.b[p];
    }
    x[idx] = xv;
    b[idx] = bv;
    if (ncol == 0) t[idx] = (T)0;
  }
  __syncthreads();

  MG_LDS T* xs = tile_smooth<T, K>(F, m, x, t, b, W, R, nsteps, ncol, omega);

  // defect on the region shrunk by H - 1 (in place into b)
  tile_defect<T, K>(F, m, xs, b, W, R, H - 1);
  __syncthreads();

  // full weighting at the coarse nodes of the tile; zero coarse start
  {
    const int ca = TX >> 1, n = ca * (TY >> 1);
    const int lo = C.py ? 0 : 1, hi = C.py ? C.ny - 1 : C.ny - 2;
    for (int idx = threadIdx.x; idx < n; idx += FT) {
      const int rb = idx / ca, a = idx - rb * ca;
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
    for (int idx = threadIdx.x; idx < n; idx += FT) {
      const int r = idx / TX;
      const int lj = H + r, li = H + idx - r * TX;
      const int gj = m.gj(lj), gi = m.gi(li);
      if (!m.unknown(gi, gj) || gj >= F.ny) continue;
      F.t[(size_t)gj * F.pitch + gi] = xs[lj * W + li];
    }
  }
}

// ------------------------------------------------------------------ post-pass

// mode: POST_PLAIN, POST_NORM (finest level: stopping test of the new
// iterate), POST_MIXED (finest FP32 level: x64 += e, e = 0).
template <typename T, int K, bool FINE>
__global__ void __launch_bounds__(FT) k_post(const Level<T>* __restrict__ Fs, const Level<T>* __restrict__ Cs, int TX,
                                             int TY, int H, int ntx, int nty, int nsteps, int ncol, T omega, int mode,
                                             const Level<double>* __restrict__ X64s) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double sh[FT / 64];
  const Level<T> F = Fs[blockIdx.z];
  SolveState* st = F.st;
  if (st->done) return;
  const Level<T> C = Cs[blockIdx.z];
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
  MG_LDS T* ec = t + (ncol == 0 ? W * R : 0);
  {
    const int clo = C.py ? 0 : 1, chi = C.py ? C.ny - 1 : C.ny - 2;
    for (int idx = threadIdx.x; idx < CW * CR; idx += FT) {
      const int r = idx / CW, c = idx - r * CW;
      const int I = cI0 + c;
      int J = cJ0 + r;
      T v = (T)0;
      if (C.py) J = ((J % C.ny) + C.ny) % C.ny;
      if (I >= 1 && I <= C.nx - 2 && J >= clo && J <= chi) v = C.x[(size_t)J * C.pitch + I];
      ec[idx] = v;
    }
  }
  __syncthreads();
  const FDiv dW(W);
  for (int idx = threadIdx.x; idx < W * R; idx += FT) {
    const int lj = dW.q(idx), li = idx - lj * W;
    const int gi = m.gi(li), gj = m.gj(lj);
    T xv = (T)0, bv = (T)0;
    if (m.unknown(gi, gj)) {
      const size_t p = (size_t)m.wrapj(gj) * F.pitch + gi;
      const int I = gi >> 1, J = gj >> 1;
      const MG_LDS T* r0 = ec + (J - cJ0) * CW + (I - cI0);
      const MG_LDS T* r1 = r0 + CW;
      xv = F.t[p] + prolong_combine(r0[0], r0[1], r1[0], r1[1], gi & 1, gj & 1);
      bv = F.b[p];
    }
    x[idx] = xv;
    b[idx] = bv;
    if (ncol == 0) t[idx] = (T)0;
  }
  __syncthreads();

  MG_LDS T* xs = tile_smooth<T, K>(F, m, x, t, b, W, R, nsteps, ncol, omega);

  double acc = 0.0;
  const int n = TX * TY;
  for (int idx = threadIdx.x; idx < n; idx += FT) {
    const int r = idx / TX;
    const int lj = H + r, li = H + idx - r * TX;
    const int gj = m.gj(lj), gi = m.gi(li);
    if (!m.unknown(gi, gj) || gj >= F.ny) continue;
    const size_t p = (size_t)gj * F.pitch + gi;
    const int q = lj * W + li;
    if (mode == POST_MIXED) {
      const Level<double>& X = X64s[blockIdx.z];
      X.x[(size_t)gj * X.pitch + gi] += (double)xs[q];
      F.x[p] = (T)0;
    } else {
      F.x[p] = xs[q];
      if (mode == POST_NORM) {
        const T d = defect_val<K>(F, LXW<T>{xs + q, W}, b[q], gi, gj, wrap_dn(gj, F.ny, F.py));
        acc += (double)d * (double)d;
      }
    }
  }
  if (mode == POST_NORM) {
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
  g.ntx = (nx + TX - 1) / TX;
  g.nty = (ny + TY - 1) / TY;
  return g;
}

template <typename T>
size_t pre_lds_bytes(const TileGeom& g, int ncol) {
  const size_t W = g.TX + 2 * g.H, R = g.TY + 2 * g.H;
  return W * R * (ncol == 0 ? 3 : 2) * sizeof(T);
}

template <typename T>
size_t post_lds_bytes(const TileGeom& g, int ncol) {
  const size_t W = g.TX + 2 * g.H, R = g.TY + 2 * g.H;
  const size_t CW = (W >> 1) + 2, CR = (R >> 1) + 2;
  return (W * R * (ncol == 0 ? 3 : 2) + CW * CR) * sizeof(T);
}

template <typename T>
hipError_t prepare_fused() {
  const void* ks[8] = {(const void*)k_pre<T, ST5, false>,  (const void*)k_pre<T, ST9, false>,
                       (const void*)k_post<T, ST5, false>, (const void*)k_post<T, ST9, false>,
                       (const void*)k_pre<T, ST5, true>,   (const void*)k_pre<T, ST9, true>,
                       (const void*)k_post<T, ST5, true>,  (const void*)k_post<T, ST9, true>};
  for (const void* k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)FUSED_LDS_MAX);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_pre(const Level<T>* Fs, const Level<T>* Cs, const TileGeom& g, int nsteps, int ncol, T omega,
                      int kind, bool fine, int nslots, hipStream_t st) {
  auto k = kind == ST5 ? (fine ? k_pre<T, ST5, true> : k_pre<T, ST5, false>)
                       : (fine ? k_pre<T, ST9, true> : k_pre<T, ST9, false>);
  hipLaunchKernelGGL(k, dim3(g.ntx * g.nty, 1, nslots), dim3(FT), pre_lds_bytes<T>(g, ncol), st, Fs, Cs, g.TX, g.TY,
                     g.H, g.ntx, g.nty, nsteps, ncol, omega);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_post(const Level<T>* Fs, const Level<T>* Cs, const TileGeom& g, int nsteps, int ncol, T omega,
                       int mode, const Level<double>* X64s, int kind, bool fine, int nslots, hipStream_t st,
                       bool with_finish) {
  auto k = kind == ST5 ? (fine ? k_post<T, ST5, true> : k_post<T, ST5, false>)
                       : (fine ? k_post<T, ST9, true> : k_post<T, ST9, false>);
  hipLaunchKernelGGL(k, dim3(g.ntx * g.nty, 1, nslots), dim3(FT), post_lds_bytes<T>(g, ncol), st, Fs, Cs, g.TX, g.TY,
                     g.H, g.ntx, g.nty, nsteps, ncol, omega, mode, X64s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || mode != POST_NORM || !with_finish) return e;
  return launch_norm_finish<T>(Fs, g.ntx * g.nty, NORM_CHECK, nslots, st);
}

#define MG_FUSED_INSTANTIATE(T)                                                                                    \
  template size_t pre_lds_bytes<T>(const TileGeom&, int);                                                          \
  template size_t post_lds_bytes<T>(const TileGeom&, int);                                                         \
  template hipError_t prepare_fused<T>();                                                                          \
  template hipError_t launch_pre<T>(const Level<T>*, const Level<T>*, const TileGeom&, int, int, T, int, bool, int, \
                                    hipStream_t);                                                                  \
  template hipError_t launch_post<T>(const Level<T>*, const Level<T>*, const TileGeom&, int, int, T, int,         \
                                     const Level<double>*, int, bool, int, hipStream_t, bool);

MG_FUSED_INSTANTIATE(double)
MG_FUSED_INSTANTIATE(float)

}  // namespace mg
