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
// node is at least r cell widths away); otherwise it widens the block.
#pragma clang fp contract(off)

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

__global__ void bbox_kernel(const double *__restrict__ xy, int n, double *__restrict__ out) {
  __shared__ double s[4][1024];
  double mnx = INFINITY, mxx = -INFINITY, mnz = INFINITY, mxz = -INFINITY;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double x = xy[2 * i], z = xy[2 * i + 1];
    mnx = fmin(mnx, x);
    mxx = fmax(mxx, x);
    mnz = fmin(mnz, z);
    mxz = fmax(mxz, z);
  }
  s[0][threadIdx.x] = mnx;
  s[1][threadIdx.x] = mxx;
  s[2][threadIdx.x] = mnz;
  s[3][threadIdx.x] = mxz;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
      s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
      s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + w]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s[0][0];
    out[1] = s[1][0];
    out[2] = s[2][0];
    out[3] = s[3][0];
  }
}

__global__ void count_kernel(const double *__restrict__ xy, int n, Grid g, int *__restrict__ cell_of,
                             int *__restrict__ count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell_z(g, xy[2 * i + 1]) * g.ncx + cell_x(g, xy[2 * i]);
  cell_of[i] = c;
  atomicAdd(&count[c], 1);
}

// Exclusive scan of `count` into start[0..n] with one 1024-thread block:
// each thread owns a contiguous chunk.
__global__ void scan_kernel(const int *__restrict__ count, int n, int *__restrict__ start) {
  __shared__ int part[1024];
  int t = threadIdx.x;
  int chunk = (n + blockDim.x - 1) / blockDim.x;
  int b = t * chunk, e = min(n, b + chunk);
  int s = 0;
  for (int i = b; i < e; ++i) s += count[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < blockDim.x; off <<= 1) {
    int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int i = b; i < e; ++i) {
    start[i] = run;
    run += count[i];
  }
  if (t == blockDim.x - 1) start[n] = part[t];
}

__global__ void scatter_kernel(const int *__restrict__ cell_of, int n, const int *__restrict__ start,
                               int *__restrict__ cursor, int *__restrict__ nodes) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell_of[i];
  int pos = start[c] + atomicAdd(&cursor[c], 1);
  nodes[pos] = i;
}

__device__ __forceinline__ bool key_less(double da, int ja, double db, int jb) {
  return da < db || (da == db && ja < jb);
}

__global__ __launch_bounds__(KNN_BLOCK) void query_kernel(
    const double *__restrict__ xy, int n_nodes, Grid g, const int *__restrict__ start,
    const int *__restrict__ cell_nodes, const int *__restrict__ centers, int n_centers,
    const int *__restrict__ n_per, int n_max, int *__restrict__ idx, int *__restrict__ err) {
  __shared__ double sd[KNN_CAP];
  __shared__ int sj[KNN_CAP];
  __shared__ int s_scan[KNN_BLOCK];
  const int q = blockIdx.x;
  const int lane = threadIdx.x;
  if (q >= n_centers) return;
  const int c = centers ? centers[q] : q;
  int nq = n_per ? n_per[q] : n_max;
  int *out = idx + static_cast<int64_t>(q) * n_max;
  if (c < 0 || c >= n_nodes || nq < 1 || nq > n_max || nq > n_nodes) {
    for (int k = lane; k < n_max; k += KNN_BLOCK) out[k] = -1;
    if (lane == 0) atomicOr(err, 1);
    return;
  }
  const double xc = xy[2 * c], zc = xy[2 * c + 1];
  const int cx = cell_x(g, xc), cz = cell_z(g, zc);
  const double smin = fmin(g.sx, g.sz);
  // first radius: enough cells for about nq nodes at the mean density
  int r = static_cast<int>(ceil(sqrt(nq / 3.14159))) ;
  if (r < 1) r = 1;
  for (int iter = 0; iter < 4096; ++iter) {
    // column range (wrapped when periodic) and row range (clamped)
    bool all_x, all_z;
    int x_lo, nxc;
    if (g.period > 0.0) {
      all_x = (2 * r + 1 >= g.ncx);
      x_lo = all_x ? 0 : cx - r;
      nxc = all_x ? g.ncx : 2 * r + 1;
    } else {
      int lo = max(0, cx - r), hi = min(g.ncx - 1, cx + r);
      all_x = (lo == 0 && hi == g.ncx - 1);
      x_lo = lo;
      nxc = hi - lo + 1;
    }
    int z_lo = max(0, cz - r), z_hi = min(g.ncz - 1, cz + r);
    all_z = (z_lo == 0 && z_hi == g.ncz - 1);
    int nzc = z_hi - z_lo + 1;
    int ncell = nxc * nzc;
    // pass 1: per-lane candidate counts
    int my = 0;
    for (int t = lane; t < ncell; t += KNN_BLOCK) {
      int ix = x_lo + t % nxc;
      if (g.period > 0.0) ix = ((ix % g.ncx) + g.ncx) % g.ncx;
      int iz = z_lo + t / nxc;
      int cc = iz * g.ncx + ix;
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
    if (total > KNN_CAP) {
      if (lane == 0) atomicOr(err, 2);
      for (int k = lane; k < n_max; k += KNN_BLOCK) out[k] = -1;
      return;
    }
    // pass 2: keys into LDS
    for (int t = lane; t < ncell; t += KNN_BLOCK) {
      int ix = x_lo + t % nxc;
      if (g.period > 0.0) ix = ((ix % g.ncx) + g.ncx) % g.ncx;
      int iz = z_lo + t / nxc;
      int cc = iz * g.ncx + ix;
      for (int p = start[cc]; p < start[cc + 1]; ++p) {
        int j = cell_nodes[p];
        sd[pos] = key_d2(xy[2 * j], xy[2 * j + 1], xc, zc, g.period);
        sj[pos] = j;
        ++pos;
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
    bool covered = all_x && all_z;
    double reach = r * smin;
    bool ok = total >= nq && (covered || sd[nq - 1] < reach * reach * (1.0 - 1e-12));
    if (ok) {
      for (int k = lane; k < n_max; k += KNN_BLOCK) out[k] = k < nq ? sj[k] : -1;
      return;
    }
    if (covered) {  // fewer nodes than nq in the whole set: cannot happen after checks
      if (lane == 0) atomicOr(err, 4);
      for (int k = lane; k < n_max; k += KNN_BLOCK) out[k] = -1;
      return;
    }
    ++r;
    __syncthreads();
  }
}

}  // namespace

int knn_run(rbffd_ctx *ctx, const rbffd_stencils *st, int32_t *idx) {
  const int n = static_cast<int>(st->n_nodes);
  const int nc = static_cast<int>(st->n_centers);
  hipStream_t s = ctx->stream;
  DevBuf d_box, d_err;
  RBFFD_HIP(ctx, d_box.alloc(4 * sizeof(double)));
  RBFFD_HIP(ctx, d_err.alloc(sizeof(int)));
  bbox_kernel<<<1, 1024, 0, s>>>(st->xy, n, d_box.as<double>());
  RBFFD_HIP(ctx, hipGetLastError());
  double box[4];
  RBFFD_HIP(ctx, hipMemcpyAsync(box, d_box.p, sizeof(box), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  if (!(std::isfinite(box[0]) && std::isfinite(box[1]) && std::isfinite(box[2]) && std::isfinite(box[3])))
    return rbffd_fail(ctx, RBFFD_EINVAL, "non-finite node coordinates");
  Grid g{};
  g.period = st->period_x;
  double lx = st->period_x > 0.0 ? st->period_x : box[1] - box[0];
  double lz = box[3] - box[2];
  if (st->period_x > 0.0 && box[1] - box[0] >= st->period_x)
    return rbffd_fail(ctx, RBFFD_EINVAL, "x extent %g not inside one period %g", box[1] - box[0], st->period_x);
  double ext = fmax(lx, lz);
  if (!(ext > 0.0)) ext = 1.0;
  double area = fmax(lx, 1e-12 * ext) * fmax(lz, 1e-12 * ext);
  double sc = sqrt(area / n);
  g.x0 = box[0];
  g.z0 = box[2];
  g.ncx = lx > 0.0 ? static_cast<int>(fmin(fmax(floor(lx / sc), 1.0), 1 << 20)) : 1;
  g.ncz = lz > 0.0 ? static_cast<int>(fmin(fmax(floor(lz / sc), 1.0), 1 << 20)) : 1;
  while (static_cast<int64_t>(g.ncx) * g.ncz > 4 * static_cast<int64_t>(n) + 16) {
    g.ncx = max(1, g.ncx / 2);
    g.ncz = max(1, g.ncz / 2);
  }
  g.sx = lx > 0.0 ? lx / g.ncx : 1.0;
  g.sz = lz > 0.0 ? lz / g.ncz : 1.0;
  const int ncell = g.ncx * g.ncz;
  DevBuf d_cellof, d_count, d_start, d_cursor, d_nodes;
  RBFFD_HIP(ctx, d_cellof.alloc(sizeof(int) * n));
  RBFFD_HIP(ctx, d_count.alloc(sizeof(int) * ncell));
  RBFFD_HIP(ctx, d_start.alloc(sizeof(int) * (ncell + 1)));
  RBFFD_HIP(ctx, d_cursor.alloc(sizeof(int) * ncell));
  RBFFD_HIP(ctx, d_nodes.alloc(sizeof(int) * n));
  RBFFD_HIP(ctx, hipMemsetAsync(d_count.p, 0, sizeof(int) * ncell, s));
  RBFFD_HIP(ctx, hipMemsetAsync(d_cursor.p, 0, sizeof(int) * ncell, s));
  RBFFD_HIP(ctx, hipMemsetAsync(d_err.p, 0, sizeof(int), s));
  count_kernel<<<grid_for(n, 256), 256, 0, s>>>(st->xy, n, g, d_cellof.as<int>(), d_count.as<int>());
  scan_kernel<<<1, 1024, 0, s>>>(d_count.as<int>(), ncell, d_start.as<int>());
  scatter_kernel<<<grid_for(n, 256), 256, 0, s>>>(d_cellof.as<int>(), n, d_start.as<int>(),
                                                  d_cursor.as<int>(), d_nodes.as<int>());
  query_kernel<<<nc, KNN_BLOCK, 0, s>>>(st->xy, n, g, d_start.as<int>(), d_nodes.as<int>(), st->centers,
                                        nc, st->n_per, st->n_max, idx, d_err.as<int>());
  RBFFD_HIP(ctx, hipGetLastError());
  int err = 0;
  RBFFD_HIP(ctx, hipMemcpyAsync(&err, d_err.p, sizeof(int), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  if (err & 1) return rbffd_fail(ctx, RBFFD_EINVAL, "bad centre index or stencil size");
  if (err & 2) return rbffd_fail(ctx, RBFFD_EINVAL, "node set too non-uniform: >%d candidates", KNN_CAP);
  if (err & 4) return rbffd_fail(ctx, RBFFD_EINVAL, "stencil larger than the node set");
  return RBFFD_OK;
}
