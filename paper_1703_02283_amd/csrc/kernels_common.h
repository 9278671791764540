// Device-side pieces shared by the product kernels: the XCD-aware tile order
// and the affine epilogue of ipr::Epilogue.
#pragma once
#include "ipr_internal.h"

namespace ipr {

struct Grid {
  int nt;     // tiles per edge
  int g;      // super-tile edge in tiles
  int s;      // super-tiles per edge
  int ntot;   // logical workgroups (super-tiles * g * g)
  int nwg;    // launched workgroups (ntot rounded up to a multiple of 8)
  int nreal;  // triangle mode: tiles with row-block <= column-block (else ntot)
};

// Tiles of super-row si in triangle mode: its diagonal super-tile's upper
// triangle and the full tiles to the right of it.
__host__ __device__ inline int tri_row_tiles(int si, int nt, int g) {
  const int rows = nt - si * g < g ? nt - si * g : g;
  const int rest = nt - (si + 1) * g;
  return rows * (rows + 1) / 2 + (rest > 0 ? rows * rest : 0);
}

inline Grid make_grid(int n, int tri, int tile) {
  Grid gr;
  gr.nt = (n + tile - 1) / tile;
  gr.g = gr.nt < 8 ? gr.nt : 8;
  gr.s = (gr.nt + gr.g - 1) / gr.g;
  const int nsuper = tri ? gr.s * (gr.s + 1) / 2 : gr.s * gr.s;
  gr.ntot = nsuper * gr.g * gr.g;
  gr.nwg = (gr.ntot + 7) / 8 * 8;
  gr.nreal = gr.ntot;
  if (tri) {
    gr.nreal = 0;
    for (int si = 0; si < gr.s; ++si) gr.nreal += tri_row_tiles(si, gr.nt, gr.g);
  }
  return gr;
}

// Workgroup w is dispatched to XCD w % 8. The logical index gives each XCD a
// contiguous run of g x g-tile super-tiles (column-major inside a super-tile),
// so the row and column panels of the tiles an XCD has in flight share its L2.
// In triangle mode super-tiles enumerate the upper triangle row by row.
__device__ __forceinline__ int logical_wg() {
  const int per = gridDim.x >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

__device__ __forceinline__ bool tile_of(int lw, const Grid& gr, int tri, int* bi, int* bj) {
  if (lw >= gr.ntot) return false;
  const int gg = gr.g * gr.g;
  const int u = lw / gg, loc = lw - u * gg;
  int si, sj;
  if (tri) {
    int r = 0, base = 0;
    while (base + (gr.s - r) <= u) {
      base += gr.s - r;
      ++r;
    }
    si = r;
    sj = r + (u - base);
  } else {
    si = u / gr.s;
    sj = u - si * gr.s;
  }
  *bi = si * gr.g + loc % gr.g;
  *bj = sj * gr.g + loc / gr.g;
  return *bi < gr.nt && *bj < gr.nt && (!tri || *bi <= *bj);
}

// Triangle mode without empty workgroups: the r-th tile with row-block <=
// column-block in the order of tile_of (super-rows in turn; in each, the
// diagonal super-tile's upper triangle column by column, then the tiles to
// its right column by column). Lets the caller give every XCD the same number
// of tiles: with whole super-tiles per XCD, a diagonal super-tile (36 tiles)
// against a full one (64) left one XCD with 12% more tiles than the mean.
__device__ __forceinline__ bool tri_tile_of(int r, const Grid& gr, int* bi, int* bj) {
  int si = 0;
  for (; si < gr.s; ++si) {
    const int cnt = tri_row_tiles(si, gr.nt, gr.g);
    if (r < cnt) break;
    r -= cnt;
  }
  if (si >= gr.s) return false;
  const int rows = gr.nt - si * gr.g < gr.g ? gr.nt - si * gr.g : gr.g;
  const int d = rows * (rows + 1) / 2;
  if (r < d) {
    int lj = 0;
    while ((lj + 1) * (lj + 2) / 2 <= r) ++lj;
    *bi = si * gr.g + r - lj * (lj + 1) / 2;
    *bj = si * gr.g + lj;
    return true;
  }
  r -= d;
  *bi = si * gr.g + r % rows;
  *bj = (si + 1) * gr.g + r / rows;
  return true;
}

// Applies the epilogue to element (i, j) whose product value is acc; adds its
// contribution to the Frobenius partial sum. kStore = false compiles out the
// approximate-storage rounding (for kernels whose callers never ask for it).
template <bool kStore = true>
__device__ __forceinline__ void epilogue_element(const Epilogue& e, int n, int tri, int i, int j,
                                                 double acc, double& psum) {
  if (i >= n || j >= n) return;
  if (tri && i > j) return;
  const size_t ij = (size_t)i * n + j;
  const size_t ji = (size_t)j * n + i;
  const bool mirror = tri && i != j;
  double v = e.alpha * acc;
  if (e.X) v += e.beta * e.X[ij];
  if (i == j) v += e.gamma;
  if (kStore && e.rfmt) v = round_store(v, e.rfmt, e.rbits);
  if (e.D) {
    e.D[ij] = v;
    if (mirror) e.D[ji] = v;
  }
  if (e.S) {
    double s = e.s_init ? ((i == j ? e.sa : 0.0) + (e.Y ? e.sb * e.Y[ij] : 0.0)) : e.S[ij];
    s += e.sc * v;
    if (kStore && e.rfmt) s = round_store(s, e.rfmt, e.rbits);
    e.S[ij] = s;
    if (mirror) e.S[ji] = s;
  }
  const double q = (i == j) ? v - e.pd : v;
  psum += mirror ? 2.0 * q * q : q * q;
}

// Sum over the workgroup's wave64s into partial[slot] (fixed order); red
// holds one double per wave.
__device__ __forceinline__ void store_partial(double* partial, int slot, double psum,
                                              double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) psum += __shfl_xor(psum, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = psum;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    partial[slot] = s;
  }
}

}  // namespace ipr
