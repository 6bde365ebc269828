// A1: stencil search -- the n nearest nodes of each centre, key (d^2, j).
//
// Section 6 builds every stencil from the n = 37 nodes nearest its centre.
// On lattices many distances tie, so the order is fixed by (d^2, j) with d^2
// evaluated as two rounded FP64 products and one rounded sum (this file is
// compiled without FMA contraction) and a minimum-image x offset for
// periodic domains. The result is exact: it equals a brute-force scan.
//
// GPU design: nodes are binned into a uniform grid of cells about one mean
// spacing wide (count, scan, scatter). One 64-lane wavefront handles one
// centre: it gathers the (d^2, j) keys of all nodes in a square block of
// cells into LDS, bitonic-sorts them, and accepts the first n_c when the
// n_c-th distance is provably inside the searched block (every unsearched
// node is at least r cell widths away); otherwise it widens the block. A
// centre whose block holds more candidates than LDS (a dense cluster) is
// finished by an exact selection kernel over the same blocks instead.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace {

constexpr int KNN_CAP = 2048;     // candidate keys held in LDS per centre
constexpr int KNN_BLOCK = 64;     // one wavefront per centre

struct Grid {
  double x0, z0, sx, sz, period;
  int ncx, ncz;
};

__device__ __forceinline__ int cell_x(const Grid &g, double x) {
  int ix = static_cast<int>(floor((x - g.x0) / g.sx));
  if (g.period > 0.0) {
    ix %= g.ncx;
    if (ix < 0) ix += g.ncx;
  } else {
    ix = ix < 0 ? 0 : (ix >= g.ncx ? g.ncx - 1 : ix);
  }
  return ix;
}

__device__ __forceinline__ int cell_z(const Grid &g, double z) {
  int iz = static_cast<int>(floor((z - g.z0) / g.sz));
  return iz < 0 ? 0 : (iz >= g.ncz ? g.ncz - 1 : iz);
}

// Squared distance exactly as specified: minimum image, then dx*dx + dz*dz
// with separate roundings (no contraction in this translation unit).
__device__ __forceinline__ double key_d2(double xj, double zj, double xc, double zc, double period) {
  double dx = xj - xc;
  if (period > 0.0) {
    double half = 0.5 * period;
    if (dx > half)
      dx = dx - period;
    else if (dx < -half)
      dx = dx + period;
  }
  double dz = zj - zc;
  double a = dx * dx;
  double b = dz * dz;
  return a + b;
}

// Bounding box in two launches: per-block partial extrema, then one block
// reduces the partials into out = {min x, max x, min z, max z}. fmin and fmax
// skip NaN operands, so a NaN coordinate is carried separately and makes
// out[0] NaN (the host rejects a non-finite box).
constexpr int BOX_THREADS = 256, BOX_BLOCKS = KNN_BOX_BLOCKS;
__global__ __launch_bounds__(BOX_THREADS) void bbox_partial_kernel(const double *__restrict__ xy, int n,
                                                                   double *__restrict__ part) {
  __shared__ double s[4][BOX_THREADS];
  double mnx = INFINITY, mxx = -INFINITY, mnz = INFINITY, mxz = -INFINITY;
  bool nan = false;
  for (int i = blockIdx.x * BOX_THREADS + threadIdx.x; i < n; i += gridDim.x * BOX_THREADS) {
    const double x = xy[2 * i], z = xy[2 * i + 1];
    nan = nan || isnan(x) || isnan(z);
    mnx = fmin(mnx, x);
    mxx = fmax(mxx, x);
    mnz = fmin(mnz, z);
    mxz = fmax(mxz, z);
  }
  s[0][threadIdx.x] = mnx;
  s[1][threadIdx.x] = mxx;
  s[2][threadIdx.x] = mnz;
  s[3][threadIdx.x] = mxz;
  nan = __syncthreads_or(nan);
  for (int w = BOX_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
      s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
      s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + w]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = (nan && threadIdx.x == 0) ? NAN : s[threadIdx.x][0];
}

__global__ __launch_bounds__(BOX_BLOCKS) void bbox_final_kernel(const double *__restrict__ part, int nb,
                                                                double *__restrict__ out) {
  __shared__ double s[4][BOX_BLOCKS];
  const int t = threadIdx.x;
  const bool nan = __syncthreads_or(t < nb && isnan(part[4 * t]));
  s[0][t] = t < nb ? part[4 * t] : INFINITY;
  s[1][t] = t < nb ? part[4 * t + 1] : -INFINITY;
  s[2][t] = t < nb ? part[4 * t + 2] : INFINITY;
  s[3][t] = t < nb ? part[4 * t + 3] : -INFINITY;
  __syncthreads();
  for (int w = BOX_BLOCKS / 2; w > 0; w >>= 1) {
    if (t < w) {
      s[0][t] = fmin(s[0][t], s[0][t + w]);
      s[1][t] = fmax(s[1][t], s[1][t + w]);
      s[2][t] = fmin(s[2][t], s[2][t + w]);
      s[3][t] = fmax(s[3][t], s[3][t + w]);
    }
    __syncthreads();
  }
  if (t < 4) out[t] = (nan && t == 0) ? NAN : s[t][0];
}

__global__ void count_kernel(const double *__restrict__ xy, int n, Grid g, int *__restrict__ count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell_z(g, xy[2 * i + 1]) * g.ncx + cell_x(g, xy[2 * i]);
  atomicAdd(&count[c], 1);
}

// Exclusive scan of count[0..n) into start[0..n] in three launches: each
// 1024-thread block sums SCAN_ITEMS consecutive counts per thread, one block
// scans the block sums, and each block then writes its own range's starts.
constexpr int SCAN_THREADS = 1024, SCAN_ITEMS = 4, SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
static_assert(SCAN_TILE == KNN_SCAN_TILE, "scratch size formula");

__device__ __forceinline__ int block_excl_scan(int v, int *s, int &total) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_THREADS; off <<= 1) {
    const int u = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += u;
    __syncthreads();
  }
  total = s[SCAN_THREADS - 1];
  const int r = s[t] - v;
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_tile_sum_kernel(const int *__restrict__ count, int n,
                                                                     int *__restrict__ tile_sum) {
  __shared__ int s[SCAN_THREADS];
  const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int v = 0;
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e) v += base + e < n ? count[base + e] : 0;
  int total;
  block_excl_scan(v, s, total);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Exclusive scan of the nt tile sums in place (each thread a contiguous
// chunk of them), and the grand total into start[n].
__global__ __launch_bounds__(SCAN_THREADS) void scan_tiles_kernel(int *__restrict__ tile_sum, int nt,
                                                                  int *__restrict__ start, int n) {
  __shared__ int s[SCAN_THREADS];
  const int chunk = (nt + SCAN_THREADS - 1) / SCAN_THREADS;
  const int b = threadIdx.x * chunk, e = min(nt, b + chunk);
  int v = 0;
  for (int i = b; i < e; ++i) v += tile_sum[i];
  int total;
  int run = block_excl_scan(v, s, total);
  for (int i = b; i < e; ++i) {
    const int c = tile_sum[i];
    tile_sum[i] = run;
    run += c;
  }
  if (threadIdx.x == 0) start[n] = total;
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_write_kernel(const int *__restrict__ count, int n,
                                                                  const int *__restrict__ tile_off,
                                                                  int *__restrict__ start) {
  __shared__ int s[SCAN_THREADS];
  const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int c[SCAN_ITEMS], v = 0;
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e) {
    c[e] = base + e < n ? count[base + e] : 0;
    v += c[e];
  }
  int total;
  int run = block_excl_scan(v, s, total) + tile_off[blockIdx.x];
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e) {
    if (base + e < n) start[base + e] = run;
    run += c[e];
  }
}

// Node i goes to its cell's range of `nodes`; count[c] (the cell's size)
// is consumed as the cursor, so the order within a cell is arbitrary (the
// query orders candidates by their keys).
__global__ void scatter_kernel(const double *__restrict__ xy, int n, Grid g, const int *__restrict__ start,
                               int *__restrict__ count, int *__restrict__ nodes) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell_z(g, xy[2 * i + 1]) * g.ncx + cell_x(g, xy[2 * i]);
  nodes[start[c] + atomicSub(&count[c], 1) - 1] = i;
}

__device__ __forceinline__ bool key_less(double da, int ja, double db, int jb) {
  return da < db || (da == db && ja < jb);
}

// The square block of cells within r of cell (cx, cz): columns x_lo ..
// x_lo + nxc - 1 (taken modulo ncx when periodic), rows z_lo .. z_lo + nzc - 1;
// `covered` when the block is the whole grid.
struct CellBlock {
  int x_lo, nxc, z_lo, nzc;
  bool covered;
};
__device__ __forceinline__ CellBlock cell_block(const Grid &g, int cx, int cz, int r) {
  CellBlock b;
  bool all_x;
  if (g.period > 0.0) {
    all_x = (2 * r + 1 >= g.ncx);
    b.x_lo = all_x ? 0 : cx - r;
    b.nxc = all_x ? g.ncx : 2 * r + 1;
  } else {
    const int lo = max(0, cx - r), hi = min(g.ncx - 1, cx + r);
    all_x = (lo == 0 && hi == g.ncx - 1);
    b.x_lo = lo;
    b.nxc = hi - lo + 1;
  }
  const int z_hi = min(g.ncz - 1, cz + r);
  b.z_lo = max(0, cz - r);
  b.nzc = z_hi - b.z_lo + 1;
  b.covered = all_x && b.z_lo == 0 && z_hi == g.ncz - 1;
  return b;
}

// Row iz of a block as one or two contiguous ranges of `nodes` (two when a
// periodic block wraps around x): [a0, b0) and [a1, b1).
__device__ __forceinline__ void block_row(const Grid &g, const CellBlock &b, int iz, const int *start, int &a0,
                                          int &b0, int &a1, int &b1) {
  const int row = iz * g.ncx;
  int lo = b.x_lo, hi = b.x_lo + b.nxc;  // [lo, hi) in unwrapped column numbers
  a1 = b1 = 0;
  if (lo < 0) {
    a1 = start[row + lo + g.ncx];
    b1 = start[row + g.ncx];
    lo = 0;
  } else if (hi > g.ncx) {
    a1 = start[row];
    b1 = start[row + hi - g.ncx];
    hi = g.ncx;
  }
  a0 = start[row + lo];
  b0 = start[row + hi];
}

// Cell t of a block, in row-major order within the block.
__device__ __forceinline__ int block_cell(const Grid &g, const CellBlock &b, int t) {
  int ix = b.x_lo + t % b.nxc;
  if (ix < 0)
    ix += g.ncx;
  else if (ix >= g.ncx)
    ix -= g.ncx;
  return (b.z_lo + t / b.nxc) * g.ncx + ix;
}

__global__ __launch_bounds__(KNN_BLOCK) void query_kernel(
    const double *__restrict__ xy, int n_nodes, Grid g, const int *__restrict__ start,
    const int *__restrict__ cell_nodes, const int *__restrict__ centers, int n_centers,
    const int *__restrict__ n_per, int n_max, int *__restrict__ idx, int *__restrict__ over,
    int *__restrict__ n_over) {
  __shared__ double sd[KNN_CAP];
  __shared__ int sj[KNN_CAP];
  __shared__ int s_scan[KNN_BLOCK];
  const int q = blockIdx.x;
  const int lane = threadIdx.x;
  if (q >= n_centers) return;
  const int c = centers ? centers[q] : q;
  const int nq = n_per ? n_per[q] : n_max;
  int *out = idx + static_cast<int64_t>(q) * n_max;
  // centres and sizes were checked before the launch
  const double xc = xy[2 * c], zc = xy[2 * c + 1];
  const int cx = cell_x(g, xc), cz = cell_z(g, zc);
  const double smin = fmin(g.sx, g.sz);
  // first radius: enough cells for about nq nodes at the mean density
  int r = static_cast<int>(ceil(sqrt(nq / 3.14159)));
  if (r < 1) r = 1;
  for (;;) {
    const CellBlock b = cell_block(g, cx, cz, r);
    const int ncb = b.nxc * b.nzc;
    // pass 1: per-lane candidate counts (lanes take cells)
    int my = 0;
    for (int t = lane; t < ncb; t += KNN_BLOCK) {
      const int cc = block_cell(g, b, t);
      my += start[cc + 1] - start[cc];
    }
    s_scan[lane] = my;
    __syncthreads();
    for (int off = 1; off < KNN_BLOCK; off <<= 1) {
      int v = lane >= off ? s_scan[lane - off] : 0;
      __syncthreads();
      s_scan[lane] += v;
      __syncthreads();
    }
    const int total = s_scan[KNN_BLOCK - 1];
    int pos = s_scan[lane] - my;
    __syncthreads();
    if (total > KNN_CAP) {  // a dense cluster: the exact fallback kernel takes this centre
      if (lane == 0) over[atomicAdd(n_over, 1)] = q;
      return;
    }
    // pass 2: keys into LDS
    for (int t = lane; t < ncb; t += KNN_BLOCK) {
      const int cc = block_cell(g, b, t);
      for (int p = start[cc]; p < start[cc + 1]; ++p, ++pos) {
        const int j = cell_nodes[p];
        sd[pos] = key_d2(xy[2 * j], xy[2 * j + 1], xc, zc, g.period);
        sj[pos] = j;
      }
    }
    int P = 1;
    while (P < total) P <<= 1;
    for (int t = total + lane; t < P; t += KNN_BLOCK) {
      sd[t] = INFINITY;
      sj[t] = 0x7fffffff;
    }
    __syncthreads();
    // bitonic sort of P keys, ascending
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = lane; i < P; i += KNN_BLOCK) {
          int l = i ^ j;
          if (l > i) {
            bool up = (i & k) == 0;
            double di = sd[i], dl = sd[l];
            int ji = sj[i], jl = sj[l];
            bool swap = up ? key_less(dl, jl, di, ji) : key_less(di, ji, dl, jl);
            if (swap) {
              sd[i] = dl;
              sd[l] = di;
              sj[i] = jl;
              sj[l] = ji;
            }
          }
        }
        __syncthreads();
      }
    }
    const double reach = r * smin;
    // covered: the block is the whole grid (holding n_nodes >= nq nodes)
    if (total >= nq && (b.covered || sd[nq - 1] < reach * reach * (1.0 - 1e-12))) {
      for (int k = lane; k < n_max; k += KNN_BLOCK) out[k] = k < nq ? sj[k] : -1;
      return;
    }
    if (b.covered) return;  // fewer nodes than nq: ruled out by the argument checks
    ++r;
    __syncthreads();
  }
}

// Centres whose block of cells held more candidates than LDS does (a dense
// cluster of nodes): the n smallest keys of the same widening blocks by
// repeated selection -- key k is the smallest key above key k - 1, found by
// a wavefront minimum over the block's nodes, which the lanes share row range
// by row range. O(n x candidates) per centre, for the few such centres.
__global__ __launch_bounds__(KNN_BLOCK) void query_wide_kernel(
    const double *__restrict__ xy, Grid g, const int *__restrict__ start, const int *__restrict__ cell_nodes,
    const int *__restrict__ centers, const int *__restrict__ n_per, int n_max, const int *__restrict__ list,
    int *__restrict__ idx) {
  __shared__ int s_out[128];
  const int q = list[blockIdx.x];
  const int lane = threadIdx.x;
  const int c = centers ? centers[q] : q;
  const int nq = n_per ? n_per[q] : n_max;
  const double xc = xy[2 * c], zc = xy[2 * c + 1];
  const int cx = cell_x(g, xc), cz = cell_z(g, zc);
  const double smin = fmin(g.sx, g.sz);
  int r = max(1, static_cast<int>(ceil(sqrt(nq / 3.14159))));
  for (;;) {
    const CellBlock b = cell_block(g, cx, cz, r);
    int my = 0;
    for (int t = 0; t < b.nzc; ++t) {
      int a0, b0, a1, b1;
      block_row(g, b, b.z_lo + t, start, a0, b0, a1, b1);
      my += (b0 - a0) + (b1 - a1);
    }
    if (my < nq) {
      if (b.covered) return;  // fewer nodes than nq: ruled out by the argument checks
      ++r;
      continue;
    }
    double pd = -1.0;  // the last selected key (pd, pj); every key is above (-1, -1)
    int pj = -1;
    for (int k = 0; k < nq; ++k) {
      double bd = INFINITY;
      int bj = 0x7fffffff;
      for (int t = 0; t < b.nzc; ++t) {
        int a0, b0, a1, b1;
        block_row(g, b, b.z_lo + t, start, a0, b0, a1, b1);
        for (int p = a0 + lane; p < b0; p += KNN_BLOCK) {
          const int j = cell_nodes[p];
          const double d = key_d2(xy[2 * j], xy[2 * j + 1], xc, zc, g.period);
          if (key_less(pd, pj, d, j) && key_less(d, j, bd, bj)) {
            bd = d;
            bj = j;
          }
        }
        for (int p = a1 + lane; p < b1; p += KNN_BLOCK) {
          const int j = cell_nodes[p];
          const double d = key_d2(xy[2 * j], xy[2 * j + 1], xc, zc, g.period);
          if (key_less(pd, pj, d, j) && key_less(d, j, bd, bj)) {
            bd = d;
            bj = j;
          }
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double od = __shfl_xor(bd, off, 64);
        const int oj = __shfl_xor(bj, off, 64);
        if (key_less(od, oj, bd, bj)) {
          bd = od;
          bj = oj;
        }
      }
      if (lane == 0) s_out[k] = bj;
      pd = bd;
      pj = bj;
    }
    const double reach = r * smin;
    if (b.covered || pd < reach * reach * (1.0 - 1e-12)) {
      __syncthreads();
      int *out = idx + static_cast<int64_t>(q) * n_max;
      for (int k = lane; k < n_max; k += KNN_BLOCK) out[k] = k < nq ? s_out[k] : -1;
      return;
    }
    ++r;
  }
}

// grid of cells about one mean spacing wide over the box, at most n + 16 cells
Grid make_grid(const double box[4], double period, int n) {
  Grid g{};
  g.period = period;
  const double lx = period > 0.0 ? period : box[1] - box[0];
  const double lz = box[3] - box[2];
  double ext = fmax(lx, lz);
  if (!(ext > 0.0)) ext = 1.0;
  const double area = fmax(lx, 1e-12 * ext) * fmax(lz, 1e-12 * ext);
  const double sc = sqrt(area / n);
  g.x0 = box[0];
  g.z0 = box[2];
  g.ncx = lx > 0.0 ? static_cast<int>(fmin(fmax(floor(lx / sc), 1.0), 1 << 20)) : 1;
  g.ncz = lz > 0.0 ? static_cast<int>(fmin(fmax(floor(lz / sc), 1.0), 1 << 20)) : 1;
  while (static_cast<int64_t>(g.ncx) * g.ncz > static_cast<int64_t>(n) + 16) {
    g.ncx = max(1, g.ncx / 2);
    g.ncz = max(1, g.ncz / 2);
  }
  g.sx = lx > 0.0 ? lx / g.ncx : 1.0;
  g.sz = lz > 0.0 ? lz / g.ncz : 1.0;
  return g;
}

}  // namespace


int knn_run(rbffd_ctx *ctx, const rbffd_stencils *st, int32_t *idx, Workspace &ws) {
  const int n = static_cast<int>(st->n_nodes);
  const int nc = static_cast<int>(st->n_centers);
  hipStream_t s = ctx->stream;
  double *d_part, *d_small;  // box partials; box[4] then two ints (overflow count, spare)
  RBFFD_WS(ctx, ws, ws.get(4 * BOX_BLOCKS, &d_part));
  RBFFD_WS(ctx, ws, ws.get(8, &d_small));
  int *d_nover = reinterpret_cast<int *>(d_small + 4);
  const int nb = std::min(BOX_BLOCKS, static_cast<int>(grid_for(n, BOX_THREADS)));
  bbox_partial_kernel<<<nb, BOX_THREADS, 0, s>>>(st->xy, n, d_part);
  bbox_final_kernel<<<1, BOX_BLOCKS, 0, s>>>(d_part, nb, d_small);
  RBFFD_HIP(ctx, hipGetLastError());
  double box[4];
  RBFFD_HIP(ctx, hipMemcpyAsync(box, d_small, sizeof(box), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  if (!(std::isfinite(box[0]) && std::isfinite(box[1]) && std::isfinite(box[2]) && std::isfinite(box[3])))
    return rbffd_fail(ctx, RBFFD_EINVAL, "non-finite node coordinates");
  if (st->period_x > 0.0 && box[1] - box[0] >= st->period_x)
    return rbffd_fail(ctx, RBFFD_EINVAL, "x extent %g not inside one period %g", box[1] - box[0], st->period_x);
  const Grid g = make_grid(box, st->period_x, n);
  const int ncell = g.ncx * g.ncz;
  const int tiles = static_cast<int>(grid_for(ncell, SCAN_TILE));
  int *d_count, *d_start, *d_tiles, *d_nodes, *d_over;
  RBFFD_WS(ctx, ws, ws.get(ncell, &d_count));
  RBFFD_WS(ctx, ws, ws.get(ncell + 1, &d_start));
  RBFFD_WS(ctx, ws, ws.get(tiles, &d_tiles));
  RBFFD_WS(ctx, ws, ws.get(n, &d_nodes));
  RBFFD_WS(ctx, ws, ws.get(std::max(nc, 1), &d_over));
  RBFFD_HIP(ctx, hipMemsetAsync(d_count, 0, sizeof(int) * ncell, s));
  RBFFD_HIP(ctx, hipMemsetAsync(d_nover, 0, sizeof(int), s));
  count_kernel<<<grid_for(n, 256), 256, 0, s>>>(st->xy, n, g, d_count);
  scan_tile_sum_kernel<<<tiles, SCAN_THREADS, 0, s>>>(d_count, ncell, d_tiles);
  scan_tiles_kernel<<<1, SCAN_THREADS, 0, s>>>(d_tiles, tiles, d_start, ncell);
  scan_write_kernel<<<tiles, SCAN_THREADS, 0, s>>>(d_count, ncell, d_tiles, d_start);
  scatter_kernel<<<grid_for(n, 256), 256, 0, s>>>(st->xy, n, g, d_start, d_count, d_nodes);
  query_kernel<<<nc, KNN_BLOCK, 0, s>>>(st->xy, n, g, d_start, d_nodes, st->centers, nc, st->n_per, st->n_max, idx,
                                        d_over, d_nover);
  RBFFD_HIP(ctx, hipGetLastError());
  int n_over = 0;
  RBFFD_HIP(ctx, hipMemcpyAsync(&n_over, d_nover, sizeof(int), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  if (n_over > 0) {
    query_wide_kernel<<<n_over, KNN_BLOCK, 0, s>>>(st->xy, g, d_start, d_nodes, st->centers, st->n_per, st->n_max,
                                                   d_over, idx);
    RBFFD_HIP(ctx, hipGetLastError());
  }
  return RBFFD_OK;
}
