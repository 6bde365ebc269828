// A2-A4: batched RBF-FD weights, one saddle-point solve per stencil.
//
// Section 3, Eq. (weights): for phi(r) = r^m (m odd) and the monomials of
// degree <= l, the weights of operator L at centre x_c are the first n
// entries of the solution of
//     [Phi P; P^T 0] [w; v] = [L phi(|x - x_j|) at x_c ; L p_q(x_c)].
// The repeated solve over all N centres is the O(n^3 N) preprocessing cost
// the paper names. Stencils are independent, and a batch may mix n, m and l:
// a counting pass bins them on the device by system size K = n + M into six
// buckets (K <= 32, 48, 64, 80, 96, 128) and fills one work queue per bucket.
// Each bucket has its own kernel, sized to its K: two systems per wavefront
// (K <= 32; a stencil whose partner differs in shape is deferred to a second
// queue and solved one per wavefront), one system per wavefront (K <= 64),
// or one 256-thread workgroup per system (K <= 128). A kernel takes its
// items from its queue either one per wavefront or workgroup, or in a
// persistent loop over a grid sized to the device; which one, and whether
// the smallest bucket pairs systems, is a per-bucket launch shape that
// rbffd_weights_tune picks by timing. Every shape computes the same bits.
//
// Per system:
//  1. offsets of the stencil nodes from the centre (minimum image in x),
//     scaled by rho = the largest offset length;
//  2. assembly of A = [Phi P; P^T 0] of size K = n + M and of B = one
//     right-hand side per operator of this PHS order (Section 5.3, Eq.
//     eqn:laplacian for Laplacian^k of r^m): [A | B] column-major in LDS in
//     the workgroup kernel, row i of A in lane i's registers in the
//     wavefront kernels;
//  3. LU with partial pivoting (FP64, or FP32 for the mixed-precision
//     variant); the wavefront kernels move no rows and take two steps per
//     pass (both pivot rows broadcast together, one rank-2 update);
//  4. back substitution, then iterative refinement: residual b - A x with A
//     and b formed in double-double arithmetic from the FP64 node
//     coordinates (so the refinement converges to the solution of the exact
//     system, not of its FP64 rounding, which for one-sided degree-5
//     stencils differs by ~5e-10), correction through the same factors,
//     until the correction is at rounding level (with FP32 factors the
//     first passes take plain FP64 residuals of the FP64 matrix, and
//     double-double ones from there on; the wavefront kernels solve for
//     the corrections in FP32);
//  5. rescaling by rho^-q (q = derivative order) and the padded row write.
//
// FP64 matrix cores on gfx950 have the same peak as the FP64 vector ALUs,
// so the factorisation is written on the vector ALUs.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.hpp"

namespace {

#ifndef RBFFD_W_THREADS
#define RBFFD_W_THREADS 256
#endif
constexpr int W_THREADS = RBFFD_W_THREADS;
constexpr int MAX_OPS = 8;

struct WOp {
  int kind, k, order;
};

struct WArgs {
  const double *xy;
  double period;
  const int *centers;
  int n_centers;
  int n_nodes;
  const int *n_per;
  int n_max;
  const int *m_per;
  int m_uni;
  const int *l_per;
  int l_uni;
  const int *idx;
  WOp ops[MAX_OPS];
  int n_ops;
  double *w;
  int *status;
  int k_cap;
  int max_iter;
  const int *list;    // the launch's queue of stencils, list[base .. base + count)
                      // (NULL: the stencils base .. base + count - 1 themselves)
  const int2 *qinfo;  // device {base, count} of the queue (NULL: {0, n_centers}); a
                      // negative base: the queue fills `list` from its end, so its
                      // entries are list[n_centers - count .. n_centers)
  int *defer;         // two systems per wavefront: stencils left to the one-system kernel
  int *n_defer;       // their count (the deferred queue's count, device)
};

// The queue a launch drains: item t is stencil list[base + t]. Launches are
// persistent or one workgroup per item; a workgroup takes items
// blockIdx.x, blockIdx.x + gridDim.x, ...
struct QueueView {
  const int *list;
  int base, count;
  __device__ __forceinline__ int stencil(int t) const { return list ? list[base + t] : base + t; }
};
__device__ __forceinline__ QueueView queue_view(const WArgs &a) {
  QueueView v{a.list, 0, a.n_centers};
  if (a.qinfo) {
    const int2 qi = *a.qinfo;
    v.count = qi.y;
    v.base = qi.x >= 0 ? qi.x : a.n_centers - qi.y;
  }
  return v;
}

__device__ __forceinline__ int n_terms(int l) { return (l + 1) * (l + 2) / 2; }

// Graded monomial order: q -> (a, b) of x^a z^b, degree d = a + b.
__device__ __forceinline__ void mono(int q, int &a, int &b) {
  int d = 0;
  while ((d + 1) * (d + 2) / 2 <= q) ++d;
  b = q - d * (d + 1) / 2;
  a = d - b;
}

__device__ __forceinline__ double ipow(double x, int p) {
  double r = 1.0;
  for (int i = 0; i < (p < 0 ? -p : p); ++i) r *= x;
  return p < 0 ? 1.0 / r : r;
}

__device__ __forceinline__ double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

// L applied to |x - x_j|^m at the centre, node offset (x, z).
__device__ double phs_rhs(int kind, int m, int k, double x, double z) {
#pragma clang fp contract(off)
  double r2 = x * x + z * z;
  if (r2 == 0.0) return 0.0;
  double r = sqrt(r2);
  switch (kind) {
    case RBFFD_DX: return -m * ipow(r, m - 2) * x;
    case RBFFD_DZ: return -m * ipow(r, m - 2) * z;
    case RBFFD_LAP: return static_cast<double>(m * m) * ipow(r, m - 2);
    case RBFFD_HYPERLAP: {
      double c = 1.0;
      for (int i = 0; i < k; ++i) c *= static_cast<double>((m - 2 * i) * (m - 2 * i));
      return c * ipow(r, m - 2 * k);
    }
    case RBFFD_DZZ:
    case RBFFD_DXX: {
      const double t = kind == RBFFD_DZZ ? z : x;   // the differentiated coordinate
      double a = m * ipow(r, m - 2);
      double b = (m >= 4) ? m * (m - 2) * ipow(r, m - 4) * t * t : m * (m - 2) * t * t / r;
      return a + b;
    }
  }
  return 0.0;
}

// L(x^a z^b) at the origin.
__device__ double poly_rhs(int kind, int k, int a, int b) {
  switch (kind) {
    case RBFFD_DX: return (a == 1 && b == 0) ? 1.0 : 0.0;
    case RBFFD_DZ: return (a == 0 && b == 1) ? 1.0 : 0.0;
    case RBFFD_LAP: return ((a == 2 && b == 0) || (a == 0 && b == 2)) ? 2.0 : 0.0;
    case RBFFD_DZZ: return (a == 0 && b == 2) ? 2.0 : 0.0;
    case RBFFD_DXX: return (a == 2 && b == 0) ? 2.0 : 0.0;
    case RBFFD_HYPERLAP: {
      if (a + b != 2 * k || (a & 1) || (b & 1)) return 0.0;
      double c = fact(k) / (fact(a / 2) * fact(k - a / 2));
      return c * fact(a) * fact(b);
    }
  }
  return 0.0;
}

// Entry (i, j) of [Phi P; P^T 0] for scaled offsets (xi, ze).
__device__ __forceinline__ double sys_entry(int i, int j, int n, int m, const double *xi,
                                            const double *ze) {
#pragma clang fp contract(off)
  if (i < n && j < n) {
    double dx = xi[i] - xi[j], dz = ze[i] - ze[j];
    return ipow(sqrt(dx * dx + dz * dz), m);
  }
  if (i < n) {
    int a, b;
    mono(j - n, a, b);
    return ipow(xi[i], a) * ipow(ze[i], b);
  }
  if (j < n) {
    int a, b;
    mono(i - n, a, b);
    return ipow(xi[j], a) * ipow(ze[j], b);
  }
  return 0.0;
}

__device__ __forceinline__ double rhs_entry(int i, int n, int m, const WOp &op, int k_eff,
                                            const double *xi, const double *ze) {
  if (i < n) return phs_rhs(op.kind, m, k_eff, xi[i], ze[i]);
  int a, b;
  mono(i - n, a, b);
  return poly_rhs(op.kind, k_eff, a, b);
}

__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}


// ---- double-double arithmetic (error-free transformations: Knuth's TwoSum,
// Dekker's product via fused multiply-add). This file is compiled without
// FP contraction, so every sum and product below is rounded as written.
struct dd {
  double hi, lo;
};
__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi), t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
// Sum without the second error-free step: the error is within a few
// 2^-104 of |a| + |b| (not of |a + b|), which is what the residual sums and
// sums of positive terms below need.
__device__ __forceinline__ dd dd_add_terms(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  s.lo += a.lo + b.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_sqr(dd a) {
  dd p = two_prod(a.hi, a.hi);
  p.lo += 2.0 * (a.hi * a.lo);
  return fast_two_sum(p.hi, p.lo);
}
// (ah + al) - (bh + bl) for offsets of distinct stencil nodes
__device__ __forceinline__ dd dd_diff(double ah, double al, double bh, double bl) {
  dd s = two_sum(ah, -bh);
  s.lo += al - bl;
  return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_div(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul_d(b, q1));
  double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul_d(b, q2));
  double q3 = r.hi / b.hi;
  dd q = fast_two_sum(q1, q2);
  return dd_add(q, dd{q3, 0.0});
}
__device__ __forceinline__ dd dd_sqrt(dd a) {
  if (!(a.hi > 0.0)) return {0.0, 0.0};
  double x = sqrt(a.hi);
  dd r = dd_sub(a, two_prod(x, x));
  return fast_two_sum(x, r.hi / (2.0 * x));
}
// r^p for odd p >= -1 given r2 = r*r and r
__device__ __forceinline__ dd dd_rpow(dd r2, dd r, int p) {
  if (p < 0) return dd_div(dd{1.0, 0.0}, r);
  dd v = r;
  for (int i = 0; i < (p - 1) / 2; ++i) v = dd_mul(v, r2);
  return v;
}
__device__ __forceinline__ dd dd_ipow(dd x, int p) {
  dd v{1.0, 0.0};
  for (int i = 0; i < p; ++i) v = dd_mul(v, x);
  return v;
}

// Entry (i, j) of [Phi P; P^T 0] in double-double from offsets (xh+xl, zh+zl).
__device__ dd sys_entry_dd(int i, int j, int n, int m, const double *xh, const double *xl, const double *zh,
                           const double *zl) {
  if (i < n && j < n) {
    const dd dx = dd_diff(xh[i], xl[i], xh[j], xl[j]);
    const dd dz = dd_diff(zh[i], zl[i], zh[j], zl[j]);
    const dd r2 = dd_add_terms(dd_sqr(dx), dd_sqr(dz));
    if (r2.hi == 0.0) return {0.0, 0.0};
    return dd_rpow(r2, dd_sqrt(r2), m);
  }
  if (i >= n && j >= n) return {0.0, 0.0};
  const int node = i < n ? i : j;
  int a, b;
  mono((i < n ? j : i) - n, a, b);
  return dd_mul(dd_ipow(dd{xh[node], xl[node]}, a), dd_ipow(dd{zh[node], zl[node]}, b));
}

// Right-hand-side entry i of operator op in double-double, node offset (x, z)
// for rows i < n.
__device__ dd rhs_dd_at(int i, int n, int m, const WOp &op, int k, dd x, dd z) {
  if (i >= n) {
    int a, b;
    mono(i - n, a, b);
    return {poly_rhs(op.kind, k, a, b), 0.0};
  }
  dd r2 = dd_add(dd_mul(x, x), dd_mul(z, z));
  if (r2.hi == 0.0) return {0.0, 0.0};
  dd r = dd_sqrt(r2);
  switch (op.kind) {
    case RBFFD_DX: return dd_mul_d(dd_mul(dd_rpow(r2, r, m - 2), x), -static_cast<double>(m));
    case RBFFD_DZ: return dd_mul_d(dd_mul(dd_rpow(r2, r, m - 2), z), -static_cast<double>(m));
    case RBFFD_LAP: return dd_mul_d(dd_rpow(r2, r, m - 2), static_cast<double>(m * m));
    case RBFFD_HYPERLAP: {
      double c = 1.0;
      for (int q = 0; q < k; ++q) c *= static_cast<double>((m - 2 * q) * (m - 2 * q));
      return dd_mul_d(dd_rpow(r2, r, m - 2 * k), c);
    }
    case RBFFD_DZZ:
    case RBFFD_DXX: {
      const dd t = op.kind == RBFFD_DZZ ? z : x;
      dd t1 = dd_mul_d(dd_rpow(r2, r, m - 2), static_cast<double>(m));
      dd t2 = dd_mul_d(dd_mul(dd_rpow(r2, r, m - 4), dd_mul(t, t)), static_cast<double>(m * (m - 2)));
      return dd_add(t1, t2);
    }
  }
  return {0.0, 0.0};
}

__device__ __forceinline__ dd rhs_entry_dd(int i, int n, int m, const WOp &op, int k, const double *xh,
                                           const double *xl, const double *zh, const double *zl) {
  return i < n ? rhs_dd_at(i, n, m, op, k, dd{xh[i], xl[i]}, dd{zh[i], zl[i]}) : rhs_dd_at(i, n, m, op, k, {}, {});
}

// Stopping rule of the iterative refinement, after a correction d computed
// from a residual, with dprev the previous correction (the first solution
// itself for the first refinement pass). The error contracts by a factor
// g ~ |d| / |dprev| per pass, so about g |d| is left after adding d: stop
// when that is below 2^-52 |x| while the corrections contract, or when d
// itself is below 2^-48 |x|.
__device__ __forceinline__ bool refined(double dm, double xm, double dprev) {
  return dm <= 0x1p-48 * xm || (dm <= 0.5 * dprev && dm * dm <= 0x1p-52 * xm * dprev);
}

template <typename T> __device__ void block_solve(const WArgs &a, double *smem, const int q) {
  const int tid = threadIdx.x;
  const int kc = a.k_cap;
  // LDS carve-up, sized by the launch's largest system kc and operator count
  double *xs = smem;                       // [n_ops][kc] solution
  double *rs = xs + a.n_ops * kc;          // [n_ops][kc] residual / correction
  double *xi = rs + a.n_ops * kc;          // [kc] scaled x offsets (FP64)
  double *ze = xi + kc;                    // [kc] scaled z offsets (FP64)
  double *xl = ze + kc;                    // [kc] low parts of the double-double x offsets
  double *zl = xl + kc;                    // [kc] low parts of the double-double z offsets
  __shared__ double s_red[5];  // rho, converged flag, max |x|, previous correction, FP64-residual flag
  __shared__ int s_piv[128];
  __shared__ int s_gl[MAX_OPS], s_kg[MAX_OPS];  // operators of the current group, their k
  __shared__ int s_flag, s_pivrow;
  __shared__ double s_pmin, s_amax, s_akk, s_pval;
  T *A = reinterpret_cast<T *>(zl + kc);   // [kc + n_ops columns][kc], column-major

  const int c = a.centers ? a.centers[q] : q;
  const int n = a.n_per ? a.n_per[q] : a.n_max;
  const int m = a.m_per ? a.m_per[q] : a.m_uni;
  const int l = a.l_per ? a.l_per[q] : a.l_uni;
  const int M = n_terms(l);
  const int K = n + M;
  double *wrow = a.w + static_cast<int64_t>(q) * a.n_max;
  const int64_t op_stride = static_cast<int64_t>(a.n_centers) * a.n_max;

  // validity (uniform for the block)
  bool bad = (c < 0 || c >= a.n_nodes || n < 1 || n > a.n_max || m < 1 || m > 15 || (m & 1) == 0 ||
              l < 0 || l > 6 || n < M || K > kc);
  if (tid == 0) s_flag = 0;
  __syncthreads();
  if (!bad) {
    for (int t = tid; t < n; t += W_THREADS) {
      int j = a.idx[static_cast<int64_t>(q) * a.n_max + t];
      if (j < 0 || j >= a.n_nodes) s_flag = 2;
    }
  }
  __syncthreads();
  if (bad || s_flag) {
    for (int o = 0; o < a.n_ops; ++o)
      for (int t = tid; t < a.n_max; t += W_THREADS) wrow[o * op_stride + t] = 0.0;
    if (tid == 0 && a.status) a.status[q] = 2;
    return;
  }

  // 1. offsets from the centre, then scale by rho
  const double xc = a.xy[2 * c], zc = a.xy[2 * c + 1];
  for (int t = tid; t < n; t += W_THREADS) {
    int j = a.idx[static_cast<int64_t>(q) * a.n_max + t];
    dd dx = two_sum(a.xy[2 * j], -xc);  // exact offset
    if (a.period > 0.0) {
      double half = 0.5 * a.period;
      double d64 = a.xy[2 * j] - xc;
      if (d64 > half)
        dx = dd_add(dx, dd{-a.period, 0.0});
      else if (d64 < -half)
        dx = dd_add(dx, dd{a.period, 0.0});
    }
    dd dz = two_sum(a.xy[2 * j + 1], -zc);
    xi[t] = dx.hi;
    xl[t] = dx.lo;
    ze[t] = dz.hi;
    zl[t] = dz.lo;
  }
  __syncthreads();
  if (tid < 64) {
    double v = 0.0;
    for (int t = tid; t < n; t += 64) {
#pragma clang fp contract(off)
      double d2 = xi[t] * xi[t] + ze[t] * ze[t];
      v = fmax(v, d2);
    }
    v = wave_max(v);
    if (tid == 0) s_red[0] = sqrt(v);
  }
  __syncthreads();
  const double rho = s_red[0];
  if (!(rho > 0.0)) {
    for (int o = 0; o < a.n_ops; ++o)
      for (int t = tid; t < a.n_max; t += W_THREADS) wrow[o * op_stride + t] = 0.0;
    if (tid == 0 && a.status) a.status[q] = 1;
    return;
  }
  for (int t = tid; t < n; t += W_THREADS) {
    const dd ex = dd_div(dd{xi[t], xl[t]}, dd{rho, 0.0}), ez = dd_div(dd{ze[t], zl[t]}, dd{rho, 0.0});
    xi[t] = ex.hi;
    xl[t] = ex.lo;
    ze[t] = ez.hi;
    zl[t] = ez.lo;
  }
  __syncthreads();

  int status = 0;
  unsigned done = 0;
  // operators grouped by PHS order: one factorisation per group
  while (done != (1u << a.n_ops) - 1u) {
    int first = 0;
    while (done & (1u << first)) ++first;
    const int mg = a.ops[first].order ? a.ops[first].order : m;
    int ng = 0;
    bool group_bad = false;
    for (int o = 0; o < a.n_ops; ++o) {
      int mo = a.ops[o].order ? a.ops[o].order : m;
      if (!(done & (1u << o)) && mo == mg) {
        const WOp &op = a.ops[o];
        const int ke = (op.kind == RBFFD_HYPERLAP && op.k == 0) ? (mg - 1) / 2 : op.k;
        if (op.kind == RBFFD_HYPERLAP && mg < 2 * ke + 1) group_bad = true;
        if (tid == 0) {
          s_gl[ng] = o;
          s_kg[ng] = ke;
        }
        ++ng;
        done |= 1u << o;
      }
    }
    __syncthreads();
    if (group_bad) {
      status = 2;
      for (int g = 0; g < ng; ++g)
        for (int t = tid; t < a.n_max; t += W_THREADS) wrow[s_gl[g] * op_stride + t] = 0.0;
      __syncthreads();
      continue;
    }
    const int Kt = K + ng;  // columns of [A | B]

    // 2. assembly, column-major: element (i, j) at j*kc + i; wavefronts take
    // columns, lanes rows
    constexpr int NW = W_THREADS / 64;
    const int wv = tid >> 6, ln = tid & 63;
    for (int j = wv; j < K; j += NW)
      for (int i = ln; i < K; i += 64) A[j * kc + i] = static_cast<T>(sys_entry(i, j, n, mg, xi, ze));
    for (int g = wv; g < ng; g += NW)
      for (int i = ln; i < K; i += 64)
        A[(K + g) * kc + i] = static_cast<T>(rhs_entry(i, n, mg, a.ops[s_gl[g]], s_kg[g], xi, ze));
    __syncthreads();
    if (tid < 64) {
      double v = 0.0;
      for (int j = 0; j < K; ++j)
        for (int i = tid; i < K; i += 64) v = fmax(v, fabs(static_cast<double>(A[j * kc + i])));
      v = wave_max(v);
      if (tid == 0) {
        s_amax = v;
        s_pmin = INFINITY;
      }
    }
    __syncthreads();

    // 3. LU with partial pivoting of [A | B]
    for (int k = 0; k < K; ++k) {
      if (tid < 64) {
        double best = -1.0;
        int bi = k;
        for (int i = k + tid; i < K; i += 64) {
          double v = fabs(static_cast<double>(A[k * kc + i]));
          if (v > best) {
            best = v;
            bi = i;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          double ob = __shfl_xor(best, off, 64);
          int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (tid == 0) {
          s_pivrow = bi;
          s_piv[k] = bi;
          s_pmin = fmin(s_pmin, best);
          s_akk = static_cast<double>(A[k * kc + k]);
          s_pval = static_cast<double>(A[k * kc + bi]);
        }
      }
      __syncthreads();
      // row interchange k <-> p in the other columns, and the multipliers of
      // column k (whose old row k now sits at row p) in the same phase
      const int p = s_pivrow;
      const T piv = static_cast<T>(s_pval), akk = static_cast<T>(s_akk);
      if (p != k) {
        for (int j = tid; j < Kt; j += W_THREADS) {
          if (j == k) continue;
          T tmp = A[j * kc + k];
          A[j * kc + k] = A[j * kc + p];
          A[j * kc + p] = tmp;
        }
      }
      const int rows = K - k - 1;
      for (int i = k + 1 + tid; i < K; i += W_THREADS) {
        const T v = i == p ? akk : A[k * kc + i];
        A[k * kc + i] = (piv != T(0)) ? v / piv : T(0);
      }
      if (tid == 0) A[k * kc + k] = piv;
      __syncthreads();
      const int cols = Kt - k - 1;
      if (rows > 0 && cols > 0) {
        const int total = rows * cols;
        int ri = tid % rows, cj = tid / rows;
        const int dq = W_THREADS / rows, dr = W_THREADS % rows;
        for (int t = tid; t < total; t += W_THREADS) {
          const int i = k + 1 + ri, j = k + 1 + cj;
          A[j * kc + i] = fma(-A[k * kc + i], A[j * kc + k], A[j * kc + i]);
          ri += dr;
          cj += dq;
          if (ri >= rows) {
            ri -= rows;
            cj += 1;
          }
        }
      }
      __syncthreads();
    }

    // 4. back substitution U x = y (y = transformed right-hand sides)
    for (int g = wv; g < ng; g += NW)
      for (int i = ln; i < K; i += 64) xs[g * kc + i] = A[(K + g) * kc + i];
    __syncthreads();
    // wavefronts take right-hand sides, lanes rows (no integer division)
    // (each right-hand side belongs to one wavefront, so its lanes read
    // x_k before lane 0 stores it, without a barrier in between)
    for (int k = K - 1; k >= 0; --k) {
      const double ukk = static_cast<double>(A[k * kc + k]);
      for (int g = wv; g < ng; g += NW) {
        const double xk = xs[g * kc + k] / ukk;
        for (int i = ln; i < k; i += 64) xs[g * kc + i] = fma(-static_cast<double>(A[k * kc + i]), xk, xs[g * kc + i]);
        if (ln == 0) xs[g * kc + k] = xk;
      }
      __syncthreads();
    }

    // 5. iterative refinement with double-double residuals (with FP32
    // factors the first passes take the FP64 entries of the assembly, as in
    // the wavefront kernels: until a correction is below 2^-24 |x| or stops
    // contracting, and without ending the refinement)
    bool converged = false;
    constexpr bool F32 = std::is_same<T, float>::value;
    bool plain = F32;  // uniform over the workgroup
    if (tid == 0) s_red[3] = -1.0;  // no previous correction yet
    for (int it = 0; it < a.max_iter && !converged; ++it) {
      // r = b - A x in double-double: 4 lanes per row, partial sums over j,
      // right-hand sides in chunks of 4 (fixed trip counts keep the
      // accumulators in registers)
      for (int g0 = 0; g0 < ng; g0 += 4) {
        const int part = tid & 3;
        for (int i = tid >> 2; i < K; i += W_THREADS / 4) {
          dd acc[4];
#pragma unroll
          for (int g = 0; g < 4; ++g) acc[g] = dd{0.0, 0.0};
          for (int j = part; j < K; j += 4) {
            const dd aij = plain ? dd{sys_entry(i, j, n, mg, xi, ze), 0.0} : sys_entry_dd(i, j, n, mg, xi, xl, ze, zl);
#pragma unroll
            for (int g = 0; g < 4; ++g)
              if (g0 + g < ng) acc[g] = dd_add_terms(acc[g], dd_mul_d(aij, xs[(g0 + g) * kc + j]));
          }
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            if (g0 + g < ng) {
              for (int off = 1; off < 4; off <<= 1) {
                dd o{__shfl_xor(acc[g].hi, off, 64), __shfl_xor(acc[g].lo, off, 64)};
                acc[g] = dd_add(acc[g], o);
              }
              if (part == 0) {
                const dd b = rhs_entry_dd(i, n, mg, a.ops[s_gl[g0 + g]], s_kg[g0 + g], xi, xl, ze, zl);
                const dd r = dd_sub(b, acc[g]);
                rs[(g0 + g) * kc + i] = r.hi + r.lo;
              }
            }
          }
        }
      }
      __syncthreads();
      if (tid < ng) {  // row interchanges, in factorisation order
        for (int k = 0; k < K; ++k) {
          int p = s_piv[k];
          if (p != k) {
            double tmp = rs[tid * kc + k];
            rs[tid * kc + k] = rs[tid * kc + p];
            rs[tid * kc + p] = tmp;
          }
        }
      }
      __syncthreads();
      for (int k = 0; k < K - 1; ++k) {  // unit lower triangle
        for (int g = wv; g < ng; g += NW)
          for (int i = k + 1 + ln; i < K; i += 64)
            rs[g * kc + i] = fma(-static_cast<double>(A[k * kc + i]), rs[g * kc + k], rs[g * kc + i]);
        __syncthreads();
      }
      for (int k = K - 1; k >= 0; --k) {  // upper triangle
        const double ukk = static_cast<double>(A[k * kc + k]);
        for (int g = wv; g < ng; g += NW) {
          const double xk = rs[g * kc + k] / ukk;
          for (int i = ln; i < k; i += 64) rs[g * kc + i] = fma(-static_cast<double>(A[k * kc + i]), xk, rs[g * kc + i]);
          if (ln == 0) rs[g * kc + k] = xk;
        }
        __syncthreads();
      }
      // x += d; converged when |d| <= 2^-48 |x| (max norms over the group)
      if (tid < 64) {
        double dmax = 0.0, xmax = 0.0;
        for (int t = 0; t < ng * 2; ++t) {
          const int g = t >> 1, i = tid + 64 * (t & 1);
          if (i >= K) continue;
          double d = rs[g * kc + i];
          double xn = xs[g * kc + i] + d;
          xs[g * kc + i] = xn;
          dmax = fmax(dmax, fabs(d));
          xmax = fmax(xmax, fabs(xn));
        }
        dmax = wave_max(dmax);
        xmax = wave_max(xmax);
        if (tid == 0) {
          const double dprev = s_red[3] >= 0.0 ? s_red[3] : xmax;
          s_red[1] = !plain && refined(dmax, xmax, dprev) ? 1.0 : 0.0;
          s_red[4] = plain && !(dmax <= 0x1p-24 * xmax || dmax > 0.5 * dprev) ? 1.0 : 0.0;
          s_red[3] = dmax;
        }
      }
      __syncthreads();
      converged = s_red[1] != 0.0;
      plain = F32 && s_red[4] != 0.0;
      __syncthreads();
    }

    // 6. status and rescaled output
    bool finite = true;
    if (tid < 64) {
      double v = 0.0;
      for (int g = 0; g < ng; ++g)
        for (int i = tid; i < K; i += 64) v = fmax(v, fabs(xs[g * kc + i]));
      v = wave_max(v);
      if (tid == 0) s_red[2] = v;
    }
    __syncthreads();
    finite = isfinite(s_red[2]);
    if (!(s_pmin >= 1e-13 * s_amax) || !converged || !finite) status = status ? status : 1;
    for (int g = 0; g < ng; ++g) {
      const WOp &op = a.ops[s_gl[g]];
      const int qd = (op.kind == RBFFD_DX || op.kind == RBFFD_DZ) ? 1
                     : (op.kind == RBFFD_HYPERLAP)                ? 2 * s_kg[g]
                                                                  : 2;
      const double scale = 1.0 / ipow(rho, qd);
      for (int t = tid; t < a.n_max; t += W_THREADS)
        wrow[s_gl[g] * op_stride + t] = (t < n && finite) ? xs[g * kc + t] * scale : 0.0;
    }
    __syncthreads();
  }
  if (tid == 0 && a.status) a.status[q] = status;
}

template <typename T>
__global__ __launch_bounds__(W_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void weights_kernel(WArgs a) {
  extern __shared__ double smem[];
  const QueueView qv = queue_view(a);
  for (int t = blockIdx.x; t < qv.count; t += gridDim.x) {
    __syncthreads();  // the previous system's LDS reads are done
    block_solve<T>(a, smem, qv.stencil(t));
  }
}

// ---- one wavefront per system, rows in registers (K <= 64) ----
//
// Lane i holds row i of A = [Phi P; P^T 0] in registers; column loops are
// unrolled over a compile-time capacity KC, so row entries have static
// register indices, and the column of a running step is one indexed register
// read in a chunk that the unrolled segment loops make static. Partial
// pivoting moves no data: the lane that supplies the pivot of step k leaves
// the active set and its row, row k of U, is broadcast through LDS (two
// steps per pass). A lane eliminated at step k keeps the eliminated entry in
// column k (no later step touches it), so its multiplier is that entry times
// 1 / pivot_k, applied in the substitutions. The right-hand sides are solved
// after the factorisation, four at a time, so registers hold one row and not
// [A | B].
//
// Iterative refinement evaluates the residual b - A x row by row with A and
// b in double-double: lane i runs over the columns j with node j's offsets
// and x_j broadcast from LDS. The first pass starts from x = 0, so the plain
// solve and the refinement share one code path.

// largest n (l + 1) with n + M(l) <= kc: entries of the power tables
__host__ __device__ constexpr int pw_cap(int kc) {
  int best = 0;
  for (int l = 0; l <= 6; ++l) {
    const int nn = kc - (l + 1) * (l + 2) / 2;
    if (nn > 0 && nn * (l + 1) > best) best = nn * (l + 1);
  }
  return best;
}

template <int KC, typename T> struct WaveShared {
  double off[KC][4];         // scaled node offsets: x hi, x lo, z hi, z lo
  double pw[pw_cap(KC)][4];  // node t, power e at t (l + 1) + e: x^e (hi, lo), z^e (hi, lo)
  double xs[KC][4];          // current solution of the right-hand sides in flight
  T prow[KC], prow2[KC];     // pivot rows of the current pair of steps
  int perm[KC];              // pivot lane of step k
  int gl[MAX_OPS], kg[MAX_OPS];  // operators of the current group, their k
};

// Product of double-doubles with an unnormalised low part (three fused
// terms): relative error within a few 2^-104.
__device__ __forceinline__ dd dd_mulr(dd a, dd b) {
  const double p = a.hi * b.hi;
  double e = fma(a.hi, b.hi, -p);
  e = fma(a.hi, b.lo, e);
  e = fma(a.lo, b.hi, e);
  return {p, e};
}

// acc + e x with the high parts summed error-free (Knuth's TwoSum) and the
// low parts in plain FP64.
__device__ __forceinline__ dd dd_acc(dd acc, dd e, double x) {
  const double p = e.hi * x;
  double pe = fma(e.hi, x, -p);
  pe = fma(e.lo, x, pe);
  const double s = acc.hi + p, bb = s - acc.hi;
  const double err = (acc.hi - (s - bb)) + (p - bb);
  return {s, acc.lo + (pe + err)};
}

// sqrt(s) for normal s > 0 within an ulp: reciprocal square root estimate,
// one Goldschmidt step and a Newton correction (no range scaling: the
// squared distances here lie between 2^-60 and 4); h returns ~1/(2 sqrt(s))
// to about 2^-40.
__device__ __forceinline__ double sqrt_pos(double s, double &h) {
  const double y0 = __builtin_amdgcn_rsq(s);
  double g = s * y0;
  h = 0.5 * y0;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  return fma(fma(-g, g, s), h, g);
}
__device__ __forceinline__ double sqrt_pos(double s) {
  double h;
  return sqrt_pos(s, h);
}

// 1 / x: hardware estimate and two Newton steps (within an ulp or two)
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recip(float x) { return 1.0f / x; }

// |a - b|^m for distinct nodes, offsets in double-double, relative error
// within about 2^-95: r^2 = s (1 + t) with s an FP64 number and t ~ 2^-52,
// y = sqrt(s) within an ulp so that s - y^2 is exact, y^m in double-double
// and (1 + t)^(m/2) to first order (the t^2 term is below 2^-100).
// MC > 0: m = MC fixed at compile time (the power fully unrolled); MC = 0:
// m at run time. Branch-free: coincident nodes (s = 0) give 0 by selection.
template <int MC = 0>
__device__ __forceinline__ dd phi_dd(const double (&a)[4], const double (&b)[4], int m) {
  if constexpr (MC > 0) m = MC;
  dd dx = two_sum(a[0], -b[0]);
  dx.lo += a[1] - b[1];
  dd dz = two_sum(a[2], -b[2]);
  dz.lo += a[3] - b[3];
  const dd px = two_prod(dx.hi, dx.hi), pz = two_prod(dz.hi, dz.hi);
  const dd s = two_sum(px.hi, pz.hi);
  double slo = s.lo + (px.lo + pz.lo);
  slo = fma(dx.hi + dx.hi, dx.lo, slo);
  slo = fma(dz.hi + dz.hi, dz.lo, slo);
  const bool pos = s.hi > 0.0;
  const double sh = pos ? s.hi : 1.0;
  double h;
  const double y = sqrt_pos(sh, h);
  const double t = (fma(-y, y, sh) + slo) * (4.0 * h * h);  // (2h)^2 ~ 1/s
  dd Y{y, 0.0};
  const dd y2 = two_prod(y, y);
  if constexpr (MC > 0) {
#pragma unroll
    for (int i = 1; i < MC; i += 2) Y = dd_mulr(Y, y2);
  } else {
    for (int i = 1; i < m; i += 2) Y = dd_mulr(Y, y2);
  }
  const double lo = fma(Y.hi * (0.5 * m), t, Y.lo);
  return {pos ? Y.hi : 0.0, pos ? lo : 0.0};
}

__device__ __forceinline__ double rl(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ __forceinline__ float rl(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Largest value over the wavefront (full exec mask): data-parallel
// primitives within rows of 16 (quad permutes, half-mirror, mirror), then the
// row broadcasts 15 and 31 carry the maximum to lane 63.
// The moved value's "old" operand is 0, the identity of an unsigned maximum
// (lanes a row mask leaves out keep it), so each step compiles to one
// v_max_u32 with a DPP source operand.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  auto step = [&](auto ctrl, auto rows) {
    const unsigned o = static_cast<unsigned>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(v), decltype(ctrl)::value, decltype(rows)::value, 0xF, false));
    v = max(v, o);
  };
  step(std::integral_constant<int, 0xB1>{}, std::integral_constant<int, 0xF>{});   // quad_perm 1,0,3,2
  step(std::integral_constant<int, 0x4E>{}, std::integral_constant<int, 0xF>{});   // quad_perm 2,3,0,1
  step(std::integral_constant<int, 0x141>{}, std::integral_constant<int, 0xF>{});  // row_half_mirror
  step(std::integral_constant<int, 0x140>{}, std::integral_constant<int, 0xF>{});  // row_mirror
  step(std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xA>{});  // row_bcast:15
  step(std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xC>{});  // row_bcast:31
  return static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
}

// Maxima over the lanes of each system when a wavefront holds H systems
// (lanes [h 64/H, (h + 1) 64/H)); every lane receives its group's value.
template <int H> __device__ __forceinline__ double group_max(double v) {
  for (int off = 32 / H; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Largest key of each group with the full exec mask: the same data-parallel
// steps as wave_max_u32; after the row broadcast 15, lane 31 holds the
// maximum of lanes 0-31 and lane 63 that of lanes 32-63.
template <int H> __device__ __forceinline__ void group_max_key(unsigned v, unsigned &k0, unsigned &k1) {
  if constexpr (H == 1) {
    k0 = k1 = wave_max_u32(v);
  } else {
    auto step = [&](auto ctrl, auto rows) {
      const unsigned o = static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), decltype(ctrl)::value,
                                                                           decltype(rows)::value, 0xF, false));
      v = max(v, o);
    };
    step(std::integral_constant<int, 0xB1>{}, std::integral_constant<int, 0xF>{});
    step(std::integral_constant<int, 0x4E>{}, std::integral_constant<int, 0xF>{});
    step(std::integral_constant<int, 0x141>{}, std::integral_constant<int, 0xF>{});
    step(std::integral_constant<int, 0x140>{}, std::integral_constant<int, 0xF>{});
    step(std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xA>{});
    k0 = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v), 31));
    k1 = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
  }
}

// Value of lane l of the own group (l wave-uniform; l0 for group 0 and l1
// for group 1 when they differ).
template <int H, typename V> __device__ __forceinline__ V group_rl(V v, int l0, int l1, int h) {
  if constexpr (H == 1) return rl(v, l0);
  const V a = rl(v, l0), b = rl(v, 32 + l1);
  return h ? b : a;
}

// One matrix row in registers, in 16-element vector chunks: static indices
// address registers directly, and a wave-uniform dynamic index k compiles to
// indexed register moves (s_set_gpr_idx_on) into chunk k / 16.
template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(16))); };
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(16))); };

// A row is held in four such chunks (local vector values, chunk j / 16 holds
// element j). They are only ever passed by value and written in the kernel
// body through RBFFD_ROW_SET, so they stay SSA values in registers; element
// stores through a pointer or reference would leave them in scratch memory.
#define RBFFD_ROW_GET(j) ((j) < 16 ? ar0[(j) & 15] : (j) < 32 ? ar1[(j) & 15] : (j) < 48 ? ar2[(j) & 15] : ar3[(j) & 15])
#define RBFFD_ROW_SET(j, x)   \
  do {                        \
    if ((j) < 16)             \
      ar0[(j) & 15] = (x);    \
    else if ((j) < 32)        \
      ar1[(j) & 15] = (x);    \
    else if ((j) < 48)        \
      ar2[(j) & 15] = (x);    \
    else                      \
      ar3[(j) & 15] = (x);    \
  } while (0)

// Element e (dynamic) of chunk c, where c is a constant once the caller's
// loops are unrolled: one indexed register read, no branch.
template <typename V>
__device__ __forceinline__ auto pickc(const V &c0, const V &c1, const V &c2, const V &c3, int c, int e) {
  auto r = c == 0 ? c0[e] : c == 1 ? c1[e] : c == 2 ? c2[e] : c3[e];
  asm volatile("" : "+v"(r));
  return r;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// State of one factorised system held by a wavefront (row `lane` of the
// factors in four chunks, eliminated entries kept), and of its stencil.
template <int KC, typename T> struct WaveRows {
  typename Vec16<T>::type c0, c1, c2, c3;
  int mystep;   // step at which this row was pivot
  int pv;       // lane k: pivot lane of step k
  double rdg;   // 1 / own pivot
};
struct WaveCtx {
  int lane, n, K, mg, P, own_pw, poly_a, poly_b;
  bool is_node, is_poly;
  dd ex, ez;  // own scaled offset
};

// Solve for the G right-hand sides of operators S.gl[g0 ..], then refine
// with double-double residuals until the stopping rule holds. Lane k of a
// system's lanes ends with unknown k in x[g]. With two systems per
// wavefront (H = 2, group h), a system that has converged keeps its
// solution while the other one refines.
//
// FP32 factors contract the error by only about cond 2^-24 per pass, so
// they take several passes. The first ones form the residual in plain FP64
// against the FP64 matrix that was rounded for the factorisation (the
// same entries, so the error still contracts, down to about cond 2^-53);
// the double-double passes start once a correction is below 2^-24 |x| or
// stops contracting, and only they may end the refinement. The switch is
// each system's own, so a system's passes do not depend on its partner in
// the wavefront (the two halves branch apart only in a pass where one has
// switched and the other not). The right-hand sides are then evaluated
// once, and so are they with FP64 factors at KC = 48 (measured: 4% faster
// there; at KC = 32 and 64 the extra registers cost more than the second
// evaluation).
template <int KC, int G, typename T, int H>
__device__ __forceinline__ void wave_refine(const WArgs &a, WaveShared<KC, T> &S, const WaveRows<KC, T> R,
                                            const WaveCtx &c, int g0, double (&x)[4], bool &converged, int h) {
  constexpr bool F32 = std::is_same<T, float>::value;
  constexpr bool KEEP_B = F32 || KC == 48;
  const int lane = c.lane, n = c.n, K = c.K, P = c.P;
  const double own[4] = {c.ex.hi, c.ex.lo, c.ez.hi, c.ez.lo};
  double dprev = 0.0;  // previous correction (the plain solution after the first pass)
  dd bc[G];            // the right-hand sides, kept over the passes (KEEP_B)
  if constexpr (KEEP_B) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int o = __builtin_amdgcn_readfirstlane(S.gl[g0 + g]);
      bc[g] = lane < K ? rhs_dd_at(lane, n, c.mg, a.ops[o], __builtin_amdgcn_readfirstlane(S.kg[g0 + g]), c.ex, c.ez)
                       : dd{0.0, 0.0};
    }
  }
  bool plain = F32;  // FP64 residuals (uniform over the system's lanes)
  for (int it = 0; it <= a.max_iter; ++it) {
    if constexpr (H == 1) {
      if (converged) break;
    } else {
      if (__ballot(!converged) == 0) break;
    }
    const bool live = !converged;
    const bool plain_pass = plain && it > 0;
    // residual b - A x in double-double (A x in plain FP64 in a plain
    // pass), rounded to FP64 (b alone when x = 0)
    dd acc[G] = {};
    if (plain_pass) {
      // the FP64 entries of the assembly: r^m = r (r^2)^((m-1)/2)
      const int e = (c.mg - 1) / 2;
      for (int j = 0; j < n; ++j) {
        const double ddx = own[0] - S.off[j][0], ddz = own[2] - S.off[j][2];
        const double s2 = ddx * ddx + ddz * ddz;
        const bool pos = s2 > 0.0;
        double r = sqrt_pos(pos ? s2 : 1.0);
        for (int t = 0; t < e; ++t) r *= s2;
        const double em = S.pw[j * P + c.poly_a][0] * S.pw[j * P + c.poly_b][2];
        const double ev = c.is_node ? (pos ? r : 0.0) : (c.is_poly ? em : 0.0);
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g].hi = fma(ev, S.xs[j][g], acc[g].hi);
      }
      int qa = 0, qb = 0;
      for (int j = n; j < K; ++j) {
        const double ev = c.is_node ? S.pw[c.own_pw + qa][0] * S.pw[c.own_pw + qb][2] : 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g].hi = fma(ev, S.xs[j][g], acc[g].hi);
        if (qa > 0) {
          --qa;
          ++qb;
        } else {
          qa = qb + 1;
          qb = 0;
        }
      }
    } else if (it > 0) {
      // node columns: Phi for node rows (0 on the diagonal), the monomials of
      // node j for polynomial rows; branch-free, with the power of r
      // unrolled for the common orders
      auto node_cols = [&](auto MC) {
        for (int j = 0; j < n; ++j) {
          const double oj[4] = {S.off[j][0], S.off[j][1], S.off[j][2], S.off[j][3]};
          const dd ep = phi_dd<decltype(MC)::value>(own, oj, c.mg);
          const double *px = S.pw[j * P + c.poly_a], *pz = S.pw[j * P + c.poly_b];
          const dd em = dd_mulr(dd{px[0], px[1]}, dd{pz[2], pz[3]});
          const dd e = c.is_node ? ep : (c.is_poly ? em : dd{0.0, 0.0});
#pragma unroll
          for (int g = 0; g < G; ++g) acc[g] = dd_acc(acc[g], e, S.xs[j][g]);
        }
      };
      switch (c.mg) {
        case 3: node_cols(std::integral_constant<int, 3>{}); break;
        case 5: node_cols(std::integral_constant<int, 5>{}); break;
        case 7: node_cols(std::integral_constant<int, 7>{}); break;
        default: node_cols(std::integral_constant<int, 0>{}); break;
      }
      // polynomial columns: the node row's own monomials
      int qa = 0, qb = 0;
      for (int j = n; j < K; ++j) {
        const double *px = S.pw[c.own_pw + qa], *pz = S.pw[c.own_pw + qb];
        const dd em = dd_mulr(dd{px[0], px[1]}, dd{pz[2], pz[3]});
        const dd e = c.is_node ? em : dd{0.0, 0.0};
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = dd_acc(acc[g], e, S.xs[j][g]);
        if (qa > 0) {
          --qa;
          ++qb;
        } else {
          qa = qb + 1;
          qb = 0;
        }
      }
    }
    double v[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      v[g] = 0.0;
      if (lane < K) {
        dd b;
        if constexpr (KEEP_B) {
          b = bc[g];
        } else {
          const int o = __builtin_amdgcn_readfirstlane(S.gl[g0 + g]);
          b = rhs_dd_at(lane, n, c.mg, a.ops[o], __builtin_amdgcn_readfirstlane(S.kg[g0 + g]), c.ex, c.ez);
        }
        const dd r = two_sum(b.hi, -acc[g].hi);
        v[g] = r.hi + (r.lo + (b.lo - acc[g].lo));
      }
    }
    // Substitutions on w = v / own pivot: every row of the factors was scaled
    // by its lane's 1 / pivot after the factorisation, so the value read from
    // the pivot lane p_k of step k is y_k / pivot_k (forward) or d_k
    // (backward) and enters each update as a scalar operand. The steps run
    // in segments of 16 (one register chunk each, unrolled), so the entry of
    // step k is an indexed read in a static chunk. They run in the factors'
    // precision: with FP32 factors the correction is only good to about
    // cond 2^-24 whatever the arithmetic, and FP32 halves the broadcasts and
    // needs no widening of the factors (the residual and x stay FP64).
    T w[G];
#pragma unroll
    for (int g = 0; g < G; ++g) w[g] = static_cast<T>(v[g] * R.rdg);
    // forward substitution L y = P v: rows not yet pivot at step k
#pragma unroll
    for (int sg = 0; sg < KC / 16; ++sg) {
      const int kend = min(16 * sg + 16, K);
      for (int k = 16 * sg; k < kend; ++k) {
        const int p0 = __builtin_amdgcn_readlane(R.pv, k), p1 = H == 1 ? p0 : __builtin_amdgcn_readlane(R.pv, 32 + k);
        const T e = pickc(R.c0, R.c1, R.c2, R.c3, sg, k & 15);
        const T lk = R.mystep > k ? e : T(0);
#pragma unroll
        for (int g = 0; g < G; ++g) w[g] = fma(-lk, group_rl<H>(w[g], p0, p1, h), w[g]);
      }
    }
    // back substitution U d = y: rows pivoted before step k
#pragma unroll
    for (int sg = KC / 16 - 1; sg >= 0; --sg) {
      const int kbeg = min(16 * sg + 15, K - 1);
      for (int k = kbeg; k >= 16 * sg; --k) {
        const int p0 = __builtin_amdgcn_readlane(R.pv, k), p1 = H == 1 ? p0 : __builtin_amdgcn_readlane(R.pv, 32 + k);
        const T e = pickc(R.c0, R.c1, R.c2, R.c3, sg, k & 15);
        const T uk = R.mystep < k ? e : T(0);
#pragma unroll
        for (int g = 0; g < G; ++g) w[g] = fma(-uk, group_rl<H>(w[g], p0, p1, h), w[g]);
      }
    }
    // lane p_k holds d_k; lane k takes it
    double dm = 0.0, xm = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const double dk = static_cast<double>(__shfl(w[g], R.pv + (64 / H) * h, 64));
      const double d = lane < K && live ? dk : 0.0;
      x[g] += d;
      dm = fmax(dm, fabs(d));
      xm = fmax(xm, fabs(x[g]));
      if (lane < K) S.xs[lane][g] = x[g];
    }
    wave_sync_lds();
    dm = group_max<H>(dm);
    xm = group_max<H>(xm);
    if (plain_pass && live && (dm <= 0x1p-24 * xm || dm > 0.5 * dprev)) plain = false;
    if (live) {
      if (!plain_pass) converged = it == 0 ? dm <= 0x1p-48 * xm : refined(dm, xm, dprev);
      dprev = dm;
    }
  }
}

// wavefronts per SIMD the register budget is fitted to (measured: with FP64
// factors, at KC = 48 three per SIMD, spilling a few values of the set-up
// and refinement code, beat two by about 2%; at KC = 64 three triple the
// time, and at KC = 32 two and four are slower than three. FP32 factors
// take half the registers for the row: three per SIMD at KC = 64 beat two
// by 16%, four at KC = 48 beat three by 7%, and four at KC = 32 gain
// nothing)
#ifndef RBFFD_WAVE_OCC64
#define RBFFD_WAVE_OCC64 2
#endif
#ifndef RBFFD_WAVE_OCC48
#define RBFFD_WAVE_OCC48 3
#endif
#ifndef RBFFD_WAVE_OCC32
#define RBFFD_WAVE_OCC32 3
#endif
#ifndef RBFFD_WAVE_OCC64F
#define RBFFD_WAVE_OCC64F 3
#endif
#ifndef RBFFD_WAVE_OCC48F
#define RBFFD_WAVE_OCC48F 4
#endif
#ifndef RBFFD_WAVE_OCC32F
#define RBFFD_WAVE_OCC32F 3
#endif
template <int KC, typename T = double> constexpr int wave_occ() {
  return std::is_same<T, float>::value
             ? (KC > 48 ? RBFFD_WAVE_OCC64F : KC > 32 ? RBFFD_WAVE_OCC48F : RBFFD_WAVE_OCC32F)
             : (KC > 48 ? RBFFD_WAVE_OCC64 : KC > 32 ? RBFFD_WAVE_OCC48 : RBFFD_WAVE_OCC32);
}


// Stencils q and r have the same n, m and l (hence the same system shape).
__device__ __forceinline__ bool same_shape(const WArgs &a, int q, int r) {
  return (!a.n_per || a.n_per[q] == a.n_per[r]) && (!a.m_per || a.m_per[q] == a.m_per[r]) &&
         (!a.l_per || a.l_per[q] == a.l_per[r]);
}

template <int KC, typename T, int H>
__device__ __forceinline__ void wave_solve(const WArgs &a, WaveShared<KC, T> (&SS)[H], const QueueView &qv,
                                           const int item) {
  static_assert(KC % 8 == 0 && KC <= 64 / H && (H == 1 || H == 2), "capacity in chunks of 8, one row per lane");
  constexpr int L = 64 / H;  // lanes per system
  const int h = H == 1 ? 0 : static_cast<int>(threadIdx.x) / L;  // the lane's system
  const int lane = static_cast<int>(threadIdx.x) % L;             // the matrix row it holds
  WaveShared<KC, T> &S = SS[h];
  // per-stencil parameters: n, m and l are wave-uniform (scalar registers)
  int q, q0;
  bool writer = true;  // this lane's system writes results (not a stand-in copy)
  if constexpr (H == 1) {
    q = __builtin_amdgcn_readfirstlane(qv.stencil(item));
    q0 = q;
  } else {
    const int i0 = 2 * item;
    q0 = __builtin_amdgcn_readfirstlane(qv.stencil(i0));
    int q1 = q0;
    if (i0 + 1 < qv.count) {
      q1 = __builtin_amdgcn_readfirstlane(qv.stencil(i0 + 1));
      if (!same_shape(a, q0, q1)) {
        if (threadIdx.x == 0) a.defer[atomicAdd(a.n_defer, 1)] = q1;
        q1 = q0;  // the upper lanes repeat system q0 without writing
      }
    }
    writer = h == 0 || q1 != q0;
    q = h ? q1 : q0;
  }
  const int c = H == 1 ? __builtin_amdgcn_readfirstlane(a.centers ? a.centers[q] : q) : (a.centers ? a.centers[q] : q);
  const int n = __builtin_amdgcn_readfirstlane(a.n_per ? a.n_per[q0] : a.n_max);
  const int m = __builtin_amdgcn_readfirstlane(a.m_per ? a.m_per[q0] : a.m_uni);
  const int l = __builtin_amdgcn_readfirstlane(a.l_per ? a.l_per[q0] : a.l_uni);
  const int M = n_terms(l);
  const int K = n + M;
  double *wrow = a.w + static_cast<int64_t>(q) * a.n_max;
  const int64_t op_stride = static_cast<int64_t>(a.n_centers) * a.n_max;
  // a pair with a system the checks below reject: both to the one-system kernel
  auto defer_pair = [&]() {
    if (lane == 0 && writer) a.defer[atomicAdd(a.n_defer, 1)] = q;
  };

  bool bad = (c < 0 || c >= a.n_nodes || n < 1 || n > a.n_max || m < 1 || m > 15 || (m & 1) == 0 || l < 0 ||
              l > 6 || n < M || K > KC);
  int node = -1;
  if (!bad && lane < n) node = a.idx[static_cast<int64_t>(q) * a.n_max + lane];
  bad = __ballot(bad || (lane < n && (node < 0 || node >= a.n_nodes))) != 0;
  if (H == 2 && bad) {
    defer_pair();
    return;
  }
  if (bad) {
    for (int o = 0; o < a.n_ops; ++o)
      for (int t = lane; t < a.n_max; t += 64) wrow[o * op_stride + t] = 0.0;
    if (lane == 0 && a.status) a.status[q] = 2;
    return;
  }

  // 1. offsets from the centre (exact double-double, minimum image in x),
  // scaled by rho = the largest offset length
  const double xc = a.xy[2 * c], zc = a.xy[2 * c + 1];
  dd dx{0.0, 0.0}, dz{0.0, 0.0};
  double d2 = 0.0;
  if (lane < n) {
    dx = two_sum(a.xy[2 * node], -xc);
    if (a.period > 0.0) {
      const double half = 0.5 * a.period, d64 = a.xy[2 * node] - xc;
      if (d64 > half)
        dx = dd_add(dx, dd{-a.period, 0.0});
      else if (d64 < -half)
        dx = dd_add(dx, dd{a.period, 0.0});
    }
    dz = two_sum(a.xy[2 * node + 1], -zc);
    d2 = dx.hi * dx.hi + dz.hi * dz.hi;
  }
  const double rho = sqrt(group_max<H>(d2));
  if (H == 2 && __ballot(!(rho > 0.0)) != 0) {
    defer_pair();
    return;
  }
  if (!(rho > 0.0)) {
    for (int o = 0; o < a.n_ops; ++o)
      for (int t = lane; t < a.n_max; t += 64) wrow[o * op_stride + t] = 0.0;
    if (lane == 0 && a.status) a.status[q] = 1;
    return;
  }
  const dd ex = lane < n ? dd_div(dx, dd{rho, 0.0}) : dd{0.0, 0.0};
  const dd ez = lane < n ? dd_div(dz, dd{rho, 0.0}) : dd{0.0, 0.0};
  const double own[4] = {ex.hi, ex.lo, ez.hi, ez.lo};
  const int P = l + 1;
  if (lane < n) {
#pragma unroll
    for (int u = 0; u < 4; ++u) S.off[lane][u] = own[u];
    dd X{1.0, 0.0}, Z{1.0, 0.0};
    for (int e = 0; e <= l; ++e) {
      double *pe = S.pw[lane * P + e];
      pe[0] = X.hi;
      pe[1] = X.lo;
      pe[2] = Z.hi;
      pe[3] = Z.lo;
      X = dd_mulr(X, ex);
      Z = dd_mulr(Z, ez);
    }
  }
  wave_sync_lds();
  const bool is_node = lane < n, is_poly = lane >= n && lane < K;
  int pa = 0, pb = 0;  // exponents of a polynomial row
  if (is_poly) mono(lane - n, pa, pb);
  const int own_pw = (is_node ? lane : 0) * P;   // own power table (node rows)
  const int poly_a = pa, poly_b = pb;

  const int n_ = n, K_ = K, P_ = P;
  int status = 0;
  unsigned done = 0;
  // operators grouped by PHS order: one factorisation per group
  while (done != (1u << a.n_ops) - 1u) {
    int first = 0;
    while (done & (1u << first)) ++first;
    const int mg = a.ops[first].order ? a.ops[first].order : m;
    int ng = 0;
    bool group_bad = false;
    for (int o = 0; o < a.n_ops; ++o) {
      const int mo = a.ops[o].order ? a.ops[o].order : m;
      if (!(done & (1u << o)) && mo == mg) {
        const WOp &op = a.ops[o];
        const int ke = (op.kind == RBFFD_HYPERLAP && op.k == 0) ? (mg - 1) / 2 : op.k;
        if (op.kind == RBFFD_HYPERLAP && mg < 2 * ke + 1) group_bad = true;
        if (lane == 0) {
          S.gl[ng] = o;
          S.kg[ng] = ke;
        }
        ++ng;
        done |= 1u << o;
      }
    }
    wave_sync_lds();
    if (group_bad) {
      status = 2;
      for (int g = 0; g < ng; ++g)
        for (int t = lane; t < a.n_max; t += L)
          if (writer) wrow[S.gl[g] * op_stride + t] = 0.0;
      continue;
    }

    // 2. row `lane` of A in FP64 (columns >= K stay zero); branch-free per
    // column: node rows take |x_i - x_j|^m or their own monomial, polynomial
    // rows the monomial of node j
    typename Vec16<T>::type ar0, ar1, ar2, ar3;
    double amax = 0.0;
    {
      // opaque copies: keeps the per-column address arithmetic inside this
      // loop instead of hoisted (and held in registers) across all groups
      int n = n_, K = K_, P = P_;
      asm volatile("" : "+s"(n), "+s"(K), "+s"(P));
      const int e = (mg - 1) / 2;  // r^m = r (r^2)^e
      int qa = 0, qb = 0;            // monomial of column j >= n, graded order
      // four columns at a time: loads and square roots first, then the
      // powers (one loop over e for all four), then the selection per row
      // kind; no branch on lanes
#pragma unroll
      for (int j0 = 0; j0 < KC; j0 += 4) {
        double r[4], r2[4], mo[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + u;
          const int jn = j < n ? j : n - 1;
          const double ddx = own[0] - S.off[jn][0], ddz = own[2] - S.off[jn][2];
          const double s2 = ddx * ddx + ddz * ddz;
          const bool pos = s2 > 0.0;
          const double y = sqrt_pos(pos ? s2 : 1.0);
          r[u] = pos ? y : 0.0;
          r2[u] = s2;
          if (j < n) {  // wave-uniform: polynomial rows take the monomials of node j
            mo[u] = S.pw[jn * P + poly_a][0] * S.pw[jn * P + poly_b][2];
          } else {      // node rows take their own monomial of column j
            mo[u] = S.pw[own_pw + qa][0] * S.pw[own_pw + qb][2];
            if (qa > 0) {
              --qa;
              ++qb;
            } else {
              qa = qb + 1;
              qb = 0;
            }
          }
        }
        for (int t = 0; t < e; ++t) {
#pragma unroll
          for (int u = 0; u < 4; ++u) r[u] *= r2[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + u;
          const double v = j < K ? (j < n ? (is_node ? r[u] : (is_poly ? mo[u] : 0.0)) : (is_node ? mo[u] : 0.0)) : 0.0;
          RBFFD_ROW_SET(j, static_cast<T>(v));
          amax = fmax(amax, fabs(v));
        }
      }
    }
    amax = group_max<H>(amax);

    // 3. LU with partial pivoting, rows stay in their lanes, two steps per
    // pass. Step k picks pivot row pa by column k; column k + 1 of every free
    // row is brought up to date with that step alone (one multiply-add with
    // row pa's entry, read from its lane), and step k + 1 picks pivot row pb
    // by it. Both pivot rows go to LDS together (row pb as it stood before
    // step k), and each free row takes both steps in one pass:
    //   a_ij -= (l_ik - l_ik1 l_pb,k) a_pa,j + l_ik1 a_pb,j    (j >= k + 2)
    // which equals step k followed by step k + 1. Column k keeps the entry
    // eliminated at step k, and column k + 1 becomes the entry eliminated at
    // step k + 1 (row pb's LDS entry there is l_pb,k a_pa,k+1, so the same
    // pass gives a_i,k+1 - l_ik a_pa,k+1). The passes run in segments of 8
    // columns: in segment s the two columns lie in chunk s / 2 and the
    // columns still to update are those from 8 s on, so the register chunk
    // and the blocks each pass reads and updates are static (the segment
    // loop is unrolled); columns up to k take zero pivot-row entries, and
    // columns >= K hold zeros in every row.
    bool fr = lane < K;  // not yet chosen as a pivot row
    int mystep = KC;     // elimination step at which this row became pivot
    double rdg = 0.0;    // 1 / own pivot
    double pmin = INFINITY;
    // largest |a_ik| over the free rows, compared on 17 mantissa bits, ties
    // to the highest lane; + 64 keeps free rows above the others
    auto pivot_key = [&](T v) {
      return ((__float_as_uint(static_cast<float>(fabs(static_cast<double>(v)))) & ~63u) + 64u) | lane;
    };
#pragma unroll
    for (int sg = 0; sg < KC / 8; ++sg) {
      const int kend = min(8 * sg + 8, K);
      for (int k = 8 * sg; k < kend; k += 2) {
        const bool two = k + 1 < K;
        // step k
        const T ck = pickc(ar0, ar1, ar2, ar3, sg / 2, k & 15);
        unsigned k0, k1;
        group_max_key<H>(fr ? pivot_key(ck) : 0u, k0, k1);
        const int pa0 = __builtin_amdgcn_readfirstlane(static_cast<int>(k0 & 63u));
        const int pa1 = __builtin_amdgcn_readfirstlane(static_cast<int>(k1 & 63u));
        const int pa = h ? pa1 : pa0;
        const T piva = group_rl<H>(ck, pa0, pa1, h);
        pmin = fmin(pmin, fabs(static_cast<double>(piva)));
        const T rpa = recip(piva);
        if (lane == pa) {
          fr = false;
          mystep = k;
          rdg = static_cast<double>(rpa);
        }
        const T la = fr ? ck * rpa : T(0);
        // column k + 1 after step k, and step k + 1
        const T c1 = pickc(ar0, ar1, ar2, ar3, sg / 2, (k + 1) & 15);
        const T ua = group_rl<H>(c1, pa0, pa1, h);
        const T c1u = fma(-la, ua, c1);
        group_max_key<H>(fr && two ? pivot_key(c1u) : 0u, k0, k1);
        const int pb0 = __builtin_amdgcn_readfirstlane(static_cast<int>(k0 & 63u));
        const int pb1 = __builtin_amdgcn_readfirstlane(static_cast<int>(k1 & 63u));
        const int pb = h ? pb1 : pb0;
        T lb = T(0), lab = T(0);
        if (two) {
          const T pivb = group_rl<H>(c1u, pb0, pb1, h);
          pmin = fmin(pmin, fabs(static_cast<double>(pivb)));
          const T rpb = recip(pivb);
          if (lane == pb) {
            fr = false;
            mystep = k + 1;
            rdg = static_cast<double>(rpb);
          }
          lb = fr ? c1u * rpb : T(0);
          lab = group_rl<H>(la, pb0, pb1, h);
        }
        // both pivot rows to LDS in the same stores
        if (lane == pa || (two && lane == pb)) {
          T *dst = lane == pa ? S.prow : S.prow2;
#pragma unroll
          for (int j = 8 * sg; j < KC; ++j) dst[j] = RBFFD_ROW_GET(j);
        }
        if (lane <= k) S.prow[lane] = T(0);
        if (lane < KC && (lane <= k + 1 || !two)) S.prow2[lane] = lane == k + 1 ? lab * ua : T(0);
        wave_sync_lds();
        const T ca = la - lb * lab;
#pragma unroll
        for (int j = 8 * sg; j < KC; ++j)
          RBFFD_ROW_SET(j, fma(-ca, S.prow[j], fma(-lb, S.prow2[j], RBFFD_ROW_GET(j))));
        wave_sync_lds();
      }
    }
    // lane k: pivot lane of step k
    if (lane < K) S.perm[mystep] = lane;
    wave_sync_lds();
    const int pv = lane < K ? S.perm[lane] : 0;
    // each row scaled by its own 1 / pivot for the substitutions
#pragma unroll
    for (int j = 0; j < KC; ++j) RBFFD_ROW_SET(j, static_cast<T>(static_cast<double>(RBFFD_ROW_GET(j)) * rdg));

    // 4. right-hand sides four at a time: solve, then refine
    for (int g0 = 0; g0 < ng; g0 += 4) {
      const int G = min(4, ng - g0);
      double x[4] = {0.0, 0.0, 0.0, 0.0};  // lane k: unknown k
      bool converged = false;
      const WaveRows<KC, T> rows{ar0, ar1, ar2, ar3, mystep, pv, rdg};
      const WaveCtx wc{lane, n, K, mg, P, own_pw, poly_a, poly_b, is_node, is_poly, ex, ez};
      switch (G) {
        case 1: wave_refine<KC, 1, T, H>(a, S, rows, wc, g0, x, converged, h); break;
        case 2: wave_refine<KC, 2, T, H>(a, S, rows, wc, g0, x, converged, h); break;
        case 3: wave_refine<KC, 3, T, H>(a, S, rows, wc, g0, x, converged, h); break;
        default: wave_refine<KC, 4, T, H>(a, S, rows, wc, g0, x, converged, h); break;
      }

      // 5. status and rescaled output
      double xmax = 0.0;
#pragma unroll
      for (int g = 0; g < 4; ++g)
        if (g < G) xmax = fmax(xmax, fabs(x[g]));
      const bool finite = isfinite(group_max<H>(xmax));
      if (!(pmin >= 1e-13 * amax) || !converged || !finite) status = status ? status : 1;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        if (g < G) {
          const int o = __builtin_amdgcn_readfirstlane(S.gl[g0 + g]);
          const WOp &op = a.ops[o];
          const int qd = (op.kind == RBFFD_DX || op.kind == RBFFD_DZ) ? 1
                         : (op.kind == RBFFD_HYPERLAP)                ? 2 * __builtin_amdgcn_readfirstlane(S.kg[g0 + g])
                                                                      : 2;
          const double scale = 1.0 / ipow(rho, qd);
          for (int t = lane; t < a.n_max; t += L)
            if (writer) wrow[o * op_stride + t] = (t < n && finite) ? x[g] * scale : 0.0;
        }
      }
    }
  }
  if (lane == 0 && writer && a.status) a.status[q] = status;
}

// H systems per wavefront: H = 1, or H = 2 for systems of up to 32 unknowns
// (lanes 0-31 and 32-63). The two systems of a wavefront have the same n, m
// and l, so every loop bound and branch on them stays wave-uniform; a
// second stencil of another shape, and a pair with an invalid or degenerate
// stencil, go to a.defer for the one-system kernel. The wavefront drains its
// share of the launch's queue (items of H systems).
template <int KC, typename T, int H = 1, bool PERSIST = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(wave_occ<KC, T>()))) void weights_wave_kernel(
    WArgs a) {
  __shared__ WaveShared<KC, T> SS[H];
  QueueView qv = queue_view(a);
  qv.base = __builtin_amdgcn_readfirstlane(qv.base);
  qv.count = __builtin_amdgcn_readfirstlane(qv.count);
  const int items = H == 2 ? (qv.count + 1) / 2 : qv.count;
  if constexpr (PERSIST) {
    for (int t = blockIdx.x; t < items; t += gridDim.x) {
      wave_sync_lds();  // the previous system's LDS reads are done
      wave_solve<KC, T, H>(a, SS, qv, t);
    }
  } else {  // one wavefront per item: no loop for the compiler to hoist work out of
    if (static_cast<int>(blockIdx.x) < items) wave_solve<KC, T, H>(a, SS, qv, blockIdx.x);
  }
}

// Launch buckets by system size: each bucket's launch reserves LDS for its
// own largest K, so small systems do not pay for the largest one.
constexpr int NBUCKET = 6;
__host__ __device__ constexpr int bucket_cap(int b) {
  return b == 0 ? 32 : b == 1 ? 48 : b == 2 ? 64 : b == 3 ? 80 : b == 4 ? 96 : 128;
}
__device__ __forceinline__ int bucket_of(int K) {
  int b = 0;
  while (b < NBUCKET - 1 && K > bucket_cap(b)) ++b;
  return b;
}

// Bucketing runs in blocks of 1024 threads: per-wavefront ballots are summed
// over the block in LDS, and each block takes one atomic per bucket
// (same-address atomics serialise, so one per wavefront cost 1.1 ms on the
// 1M-stencil batch).
constexpr int BK_BLOCK = 1024;
constexpr int BK_WAVES = BK_BLOCK / 64;

// Bucket of stencil q and its system size K, or NBUCKET (K = 0) when its n
// or l is invalid.
__device__ __forceinline__ int stencil_bucket(const int *n_per, int n_max, const int *l_per, int l_uni, int q,
                                              int &K) {
  const int n = n_per ? n_per[q] : n_max;
  const int l = l_per ? l_per[q] : l_uni;
  K = 0;
  if (l < 0 || l > 6 || n < 1 || n > n_max) return NBUCKET;
  K = n + n_terms(l);
  return bucket_of(K);
}

// count[b] and the largest K kmax[b] of each bucket b; count[NBUCKET]
// counts the stencils with an invalid n or l.
__global__ __launch_bounds__(BK_BLOCK) void bucket_count_kernel(const int *n_per, int n_max, const int *l_per,
                                                                int l_uni, int nc, int *count, int *kmax) {
  __shared__ int s_cnt[BK_WAVES][NBUCKET + 1], s_km[BK_WAVES][NBUCKET + 1];
  const int q = static_cast<int>(blockIdx.x) * BK_BLOCK + static_cast<int>(threadIdx.x);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int K = 0;
  const int b = q < nc ? stencil_bucket(n_per, n_max, l_per, l_uni, q, K) : -1;
  for (int bb = 0; bb <= NBUCKET; ++bb) {
    const uint64_t mask = __ballot(b == bb);
    int km = b == bb ? K : 0;
    for (int off = 32; off > 0; off >>= 1) km = max(km, __shfl_xor(km, off, 64));
    if (lane == 0) {
      s_cnt[wv][bb] = __popcll(mask);
      s_km[wv][bb] = km;
    }
  }
  __syncthreads();
  if (threadIdx.x <= NBUCKET) {
    int c = 0, km = 0;
    for (int w = 0; w < BK_WAVES; ++w) {
      c += s_cnt[w][threadIdx.x];
      km = max(km, s_km[w][threadIdx.x]);
    }
    if (c) {
      atomicAdd(&count[threadIdx.x], c);
      atomicMax(&kmax[threadIdx.x], km);
    }
  }
}

// cursor[b] starts at bucket b's offset in `list`. Each block reserves one
// run per bucket and fills it in ascending stencil order, so stencils that
// are neighbours in memory stay neighbours in a launch. In the run of the
// K <= 32 bucket, whose systems are solved two per wavefront, stencils of
// one shape (n, m, l) are made adjacent (by shape, then stencil) when the
// block holds more than one shape. Every stencil is valid here (the count
// rejects a batch with invalid ones).
__global__ __launch_bounds__(BK_BLOCK) void bucket_fill_kernel(const int *n_per, int n_max, const int *m_per,
                                                               int m_uni, const int *l_per, int l_uni, int nc,
                                                               int *cursor, int *list) {
  __shared__ int s_cnt[BK_WAVES][NBUCKET], s_base[NBUCKET];
  __shared__ unsigned s_key[BK_BLOCK];
  const int q = static_cast<int>(blockIdx.x) * BK_BLOCK + static_cast<int>(threadIdx.x);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int K = 0;
  const int b = q < nc ? stencil_bucket(n_per, n_max, l_per, l_uni, q, K) : -1;
  uint64_t mine = 0;
  for (int bb = 0; bb < NBUCKET; ++bb) {
    const uint64_t mask = __ballot(b == bb);
    if (lane == 0) s_cnt[wv][bb] = __popcll(mask);
    if (b == bb) mine = mask;
  }
  // shape key of a K <= 32 stencil (n < 64, l <= 6, m <= 15), else all ones
  unsigned key = 0xFFFFFFFFu;
  if (b == 0) {
    const unsigned n = static_cast<unsigned>(n_per ? n_per[q] : n_max);
    const unsigned m = static_cast<unsigned>(m_per ? m_per[q] : m_uni) & 15u;
    const unsigned l = static_cast<unsigned>(l_per ? l_per[q] : l_uni);
    key = ((n | (l << 6) | (m << 9)) << 10) | threadIdx.x;
  }
  __syncthreads();
  if (threadIdx.x < NBUCKET) {
    int t = 0;
    for (int w = 0; w < BK_WAVES; ++w) t += s_cnt[w][threadIdx.x];
    s_base[threadIdx.x] = t ? atomicAdd(&cursor[threadIdx.x], t) : 0;
  }
  // more than one shape in this block's K <= 32 run: sort the run's keys
  const unsigned shape = b == 0 ? key >> 10 : 0u;
  if (b == 0) s_key[0] = shape;  // any one of the run's shapes
  __syncthreads();
  const bool mixed = __syncthreads_or(b == 0 && shape != s_key[0]);
  if (mixed) {
    s_key[threadIdx.x] = key;
    __syncthreads();
    for (int size = 2; size <= BK_BLOCK; size <<= 1)  // bitonic sort, ascending
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        const int t = threadIdx.x, u = t ^ stride;
        if (u > t) {
          const unsigned x = s_key[t], y = s_key[u];
          if ((x > y) == ((t & size) == 0)) {
            s_key[t] = y;
            s_key[u] = x;
          }
        }
        __syncthreads();
      }
    // the run's stencils are now the first entries, by shape, then stencil
    const unsigned k = s_key[threadIdx.x];
    if (k != 0xFFFFFFFFu)
      list[s_base[0] + static_cast<int>(threadIdx.x)] = static_cast<int>(blockIdx.x) * BK_BLOCK + static_cast<int>(k & 1023u);
  }
  if ((b > 0 && b < NBUCKET) || (b == 0 && !mixed)) {
    int base = s_base[b];
    for (int w = 0; w < wv; ++w) base += s_cnt[w][b];
    list[base + __popcll(mine & ((uint64_t(1) << lane) - 1))] = q;
  }
}

// Stencils whose FP32-factorisation refinement stalled (status 1), for an
// FP64 solve: systems of up to 64 unknowns into the front of `list` (queue
// lo), larger ones into its end (queue hi); the queues' counts grow here.
__global__ void stalled_list_kernel(const int *status, const int *n_per, int n_max, const int *l_per, int l_uni,
                                    int nc, int *list, int2 *lo, int2 *hi) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc || status[q] != 1) return;
  const int K = (n_per ? n_per[q] : n_max) + n_terms(l_per ? l_per[q] : l_uni);
  if (K <= 64)
    list[atomicAdd(&lo->y, 1)] = q;
  else
    list[nc - 1 - atomicAdd(&hi->y, 1)] = q;
}

// Stencils of both stalled queues that the FP64 solve did solve: status 3.
__global__ void mark_fallback_kernel(int *status, const int *list, int nc, const int2 *lo, const int2 *hi) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc) return;
  const bool in = t < lo->y || t >= nc - hi->y;
  if (in && status[list[t]] == 0) status[list[t]] = 3;
}

__global__ void count_status_kernel(const int *status, int nc, int *counts) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  int s = status[q];
  if (s == 1) atomicAdd(&counts[0], 1);
  if (s == 2) atomicAdd(&counts[1], 1);
}

// Launch shapes of the solve kernels, chosen per size bucket by
// rbffd_weights_tune. Wavefront buckets: one wavefront per queue item, or a
// persistent grid of as many wavefronts as the compute units hold at the
// kernel's occupancy, each draining items in turn; for systems of up to 32
// unknowns also two systems per wavefront or one. Block buckets: one
// workgroup per system or 1, 2, 4 persistent workgroups per compute unit. A
// shape never changes a system's arithmetic.
struct WShape {
  bool persist, pair;
};
constexpr WShape kWaveShapes[] = {{false, true}, {true, true}, {false, false}, {true, false}};
constexpr int kBlockShapes[] = {0, 1, 2, 4};
constexpr int shape_count(int b) { return b == 0 ? 4 : b <= 2 ? 2 : 4; }
constexpr int MAX_SHAPES = 4;

// Count array layout (device, int): bucket counts and the invalid count,
// largest K per bucket, fill cursors, queues {base, count} (the six buckets,
// the stencils the pair kernel defers, the stalled systems of up to 64 and
// of more unknowns), status counts.
constexpr int Q_DEFER = NBUCKET, Q_STALL_LO = NBUCKET + 1, Q_STALL_HI = NBUCKET + 2, NQUEUE = NBUCKET + 3;
constexpr int C_KMAX = NBUCKET + 1, C_CURSOR = 2 * NBUCKET + 1, C_Q = 3 * NBUCKET + 2,
              C_STATUS = C_Q + 2 * NQUEUE, C_ALL = C_STATUS + 2;
static_assert(C_Q % 2 == 0, "queues are int2");
static_assert(C_ALL == WEIGHTS_COUNTS, "scratch size formula");

inline unsigned grid_of(int64_t items, int per_cu, int n_cu) {
  const int64_t g = per_cu > 0 ? std::min<int64_t>(items, static_cast<int64_t>(per_cu) * n_cu) : items;
  return static_cast<unsigned>(std::max<int64_t>(g, 1));
}

// A wavefront-bucket launch: one wavefront per item, or persistent (the
// compute units' resident wavefronts at the kernel's occupancy).
template <int KC, typename T, int H>
void launch_wave(const WArgs &a, int64_t items, bool persist, int n_cu, hipStream_t s) {
  if (persist)
    weights_wave_kernel<KC, T, H, true><<<grid_of(items, 4 * wave_occ<KC, T>(), n_cu), 64, 0, s>>>(a);
  else
    weights_wave_kernel<KC, T, H, false><<<grid_of(items, 0, n_cu), 64, 0, s>>>(a);
}

template <typename T> int launch_block(rbffd_ctx *ctx, const WArgs &a, int cap, int n_ops, unsigned grid) {
  const size_t head = sizeof(double) * (2 * static_cast<size_t>(n_ops) * cap + 4 * static_cast<size_t>(cap));
  const size_t lds = head + sizeof(T) * static_cast<size_t>(cap) * (cap + n_ops);
  if (lds > 156 * 1024) return rbffd_fail(ctx, RBFFD_EINVAL, "system size %d too large for LDS", cap);
  RBFFD_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&weights_kernel<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  weights_kernel<T><<<grid, W_THREADS, lds, ctx->stream>>>(a);
  return RBFFD_OK;
}

}  // namespace

int weights_run(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops, int precision,
                const int32_t *idx, double *w, int32_t *status, int32_t *n_bad, Workspace &ws, const int *shapes,
                hipEvent_t *bucket_ev) {
  hipStream_t s = ctx->stream;
  const int nc = static_cast<int>(st->n_centers);
  const int n_cu = ctx->n_cu;
  if (!shapes) shapes = ctx->wshape;
  int *d_cnt, *d_list;
  RBFFD_WS(ctx, ws, ws.get(C_ALL, &d_cnt));
  RBFFD_WS(ctx, ws, ws.get(std::max(nc, 1), &d_list));
  RBFFD_HIP(ctx, hipMemsetAsync(d_cnt, 0, C_ALL * sizeof(int), s));
  // stencils bucketed by K (and the invalid ones counted)
  bucket_count_kernel<<<grid_for(nc, BK_BLOCK), BK_BLOCK, 0, s>>>(st->n_per, st->n_max, st->l_per, st->l_uniform,
                                                                  nc, d_cnt, d_cnt + C_KMAX);
  RBFFD_HIP(ctx, hipGetLastError());
  int cnt[C_ALL];  // counts (and the invalid count), largest K per bucket, cursors, queues
  RBFFD_HIP(ctx, hipMemcpyAsync(cnt, d_cnt, C_CURSOR * sizeof(int), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  // n and l were checked before anything was written; this is a safeguard
  if (cnt[NBUCKET] > 0) return rbffd_fail(ctx, RBFFD_EINVAL, "%d stencils with invalid n or l", cnt[NBUCKET]);
  int kc = 0, n_small = 0, n_large = 0;
  for (int b = 0; b < NBUCKET; ++b) {
    kc = std::max(kc, cnt[C_KMAX + b]);
    (b <= 2 ? n_small : n_large) += cnt[b];
  }
  if (kc > 128) return rbffd_fail(ctx, RBFFD_EINVAL, "system size %d above 128", kc);

  int32_t *st_out = status;
  if (!st_out) RBFFD_WS(ctx, ws, ws.get(nc, &st_out));
  // queues: bucket b at its prefix offset in the list (its fill cursor starts
  // there), the deferred and stalled queues empty
  for (int b = 0, off = 0; b < NBUCKET; ++b) {
    cnt[C_CURSOR + b] = off;
    cnt[C_Q + 2 * b] = off;
    cnt[C_Q + 2 * b + 1] = cnt[b];
    off += cnt[b];
  }
  for (int q = NBUCKET; q < NQUEUE; ++q) {
    cnt[C_Q + 2 * q] = q == Q_STALL_HI ? -1 : 0;
    cnt[C_Q + 2 * q + 1] = 0;
  }
  RBFFD_HIP(ctx, hipMemcpyAsync(d_cnt + C_CURSOR, cnt + C_CURSOR, (C_STATUS - C_CURSOR) * sizeof(int),
                                hipMemcpyHostToDevice, s));
  bucket_fill_kernel<<<grid_for(nc, BK_BLOCK), BK_BLOCK, 0, s>>>(st->n_per, st->n_max, st->m_per, st->m_uniform,
                                                                 st->l_per, st->l_uniform, nc, d_cnt + C_CURSOR,
                                                                 d_list);
  RBFFD_HIP(ctx, hipGetLastError());
  int2 *queue = reinterpret_cast<int2 *>(d_cnt + C_Q);

  WArgs a{};
  a.xy = st->xy;
  a.period = st->period_x;
  a.centers = st->centers;
  a.n_centers = nc;
  a.n_nodes = static_cast<int>(st->n_nodes);
  a.n_per = st->n_per;
  a.n_max = st->n_max;
  a.m_per = st->m_per;
  a.m_uni = st->m_uniform;
  a.l_per = st->l_per;
  a.l_uni = st->l_uniform;
  a.idx = idx;
  for (int i = 0; i < n_ops; ++i) a.ops[i] = WOp{ops[i].kind, ops[i].k, ops[i].phs_order};
  a.n_ops = n_ops;
  a.w = w;
  a.status = st_out;
  a.max_iter = precision == RBFFD_SOLVE_FP64 ? 3 : 30;
  a.list = d_list;
  const bool f64 = precision == RBFFD_SOLVE_FP64;
  int *d_def = nullptr;
  if (cnt[0] > 0) RBFFD_WS(ctx, ws, ws.get(cnt[0], &d_def));
  for (int b = 0; b < NBUCKET; ++b) {
    if (bucket_ev) RBFFD_HIP(ctx, hipEventRecord(bucket_ev[2 * b], s));
    if (cnt[b] > 0) {
      a.qinfo = queue + b;
      a.k_cap = cnt[C_KMAX + b];  // the bucket's largest K
      if (b == 0) {
        // systems of up to 32 unknowns: two per wavefront, then the stencils
        // that kernel defers (a shape other than its partner's, a degenerate
        // one) one per wavefront, persistent over their device-counted queue;
        // or all one per wavefront
        const WShape sh = kWaveShapes[shapes[0]];
        if (sh.pair) {
          WArgs p = a;
          p.defer = d_def;
          p.n_defer = &queue[Q_DEFER].y;
          f64 ? launch_wave<32, double, 2>(p, (cnt[0] + 1) / 2, sh.persist, n_cu, s)
              : launch_wave<32, float, 2>(p, (cnt[0] + 1) / 2, sh.persist, n_cu, s);
          WArgs f = a;
          f.list = d_def;
          f.qinfo = queue + Q_DEFER;
          f64 ? launch_wave<32, double, 1>(f, cnt[0], true, n_cu, s) : launch_wave<32, float, 1>(f, cnt[0], true, n_cu, s);
        } else {
          f64 ? launch_wave<32, double, 1>(a, cnt[0], sh.persist, n_cu, s)
              : launch_wave<32, float, 1>(a, cnt[0], sh.persist, n_cu, s);
        }
      } else if (b <= 2) {  // systems of up to 64 unknowns: one wavefront each
        const bool persist = kWaveShapes[shapes[b]].persist;
        if (b == 1)
          f64 ? launch_wave<48, double, 1>(a, cnt[b], persist, n_cu, s)
              : launch_wave<48, float, 1>(a, cnt[b], persist, n_cu, s);
        else
          f64 ? launch_wave<64, double, 1>(a, cnt[b], persist, n_cu, s)
              : launch_wave<64, float, 1>(a, cnt[b], persist, n_cu, s);
      } else {  // one 256-thread workgroup per system
        const unsigned g = grid_of(cnt[b], kBlockShapes[shapes[b]], n_cu);
        const int rc = f64 ? launch_block<double>(ctx, a, a.k_cap, n_ops, g) : launch_block<float>(ctx, a, a.k_cap, n_ops, g);
        if (rc) return rc;
      }
      RBFFD_HIP(ctx, hipGetLastError());
    }
    if (bucket_ev) RBFFD_HIP(ctx, hipEventRecord(bucket_ev[2 * b + 1], s));
  }
  // FP32 factorisation: the stencils whose refinement stalled are solved
  // again in FP64 (the same kernels, over the stalled queues) and marked 3
  if (!f64) {
    int *d_fl;
    RBFFD_WS(ctx, ws, ws.get(nc, &d_fl));
    stalled_list_kernel<<<grid_for(nc, 256), 256, 0, s>>>(st_out, st->n_per, st->n_max, st->l_per, st->l_uniform, nc,
                                                          d_fl, queue + Q_STALL_LO, queue + Q_STALL_HI);
    WArgs f = a;
    f.max_iter = 3;  // the FP64 setting
    f.list = d_fl;
    if (n_small > 0) {
      f.qinfo = queue + Q_STALL_LO;
      f.k_cap = 64;
      launch_wave<64, double, 1>(f, n_small, true, n_cu, s);
    }
    if (n_large > 0) {
      f.qinfo = queue + Q_STALL_HI;
      f.k_cap = kc;
      const int rc = launch_block<double>(ctx, f, kc, n_ops, grid_of(n_large, 2, n_cu));
      if (rc) return rc;
    }
    mark_fallback_kernel<<<grid_for(nc, 256), 256, 0, s>>>(st_out, d_fl, nc, queue + Q_STALL_LO, queue + Q_STALL_HI);
    RBFFD_HIP(ctx, hipGetLastError());
  }
  count_status_kernel<<<grid_for(nc, 256), 256, 0, s>>>(st_out, nc, d_cnt + C_STATUS);
  RBFFD_HIP(ctx, hipGetLastError());
  int hk[2];
  RBFFD_HIP(ctx, hipMemcpyAsync(hk, d_cnt + C_STATUS, sizeof(hk), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  *n_bad = hk[1] > 0 ? -hk[1] : hk[0];
  return RBFFD_OK;
}

int weights_shape_count(int bucket) { return bucket >= 0 && bucket < NBUCKET ? shape_count(bucket) : 0; }

int weights_tune(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops, int precision,
                 const int32_t *idx, double *w, int32_t *status, int32_t *n_bad, int32_t *shapes, double *ms) {
  int forced[NBUCKET], best[NBUCKET], cur[NBUCKET];
  double best_ms[NBUCKET];
  for (int b = 0; b < NBUCKET; ++b) {
    forced[b] = shapes ? shapes[b] : -1;
    if (forced[b] >= shape_count(b))
      return rbffd_fail(ctx, RBFFD_EINVAL, "shape %d of bucket %d outside 0..%d", forced[b], b, shape_count(b) - 1);
    best[b] = forced[b] >= 0 ? forced[b] : ctx->wshape[b];
    best_ms[b] = -1.0;
  }
  hipEvent_t ev[2 * NBUCKET] = {};
  for (auto &e : ev) RBFFD_HIP(ctx, hipEventCreate(&e));
  int rc = RBFFD_OK;
  // every shape twice, the faster time kept: the first launch of the first
  // shape also pays for cold caches and code loading
  for (int trial_sh = 0; trial_sh < 2 * MAX_SHAPES && rc == RBFFD_OK; ++trial_sh) {
    const int sh = trial_sh % MAX_SHAPES;
    bool any = false;
    for (int b = 0; b < NBUCKET; ++b) {
      const bool trial = forced[b] < 0 && sh < shape_count(b);
      cur[b] = trial ? sh : best[b];
      any = any || trial || (forced[b] >= 0 && sh == 0);
    }
    if (!any) continue;
    Workspace ws;
    rc = weights_run(ctx, st, ops, n_ops, precision, idx, w, status, n_bad, ws, cur, ev);
    for (int b = 0; b < NBUCKET && rc == RBFFD_OK; ++b) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, ev[2 * b], ev[2 * b + 1]) != hipSuccess) continue;
      if ((forced[b] < 0 && sh < shape_count(b)) || (forced[b] >= 0 && sh == 0)) {
        if (best_ms[b] < 0.0 || t < best_ms[b]) {
          best_ms[b] = t;
          best[b] = cur[b];
        }
      }
    }
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (rc) return rc;
  for (int b = 0; b < NBUCKET; ++b) {
    ctx->wshape[b] = best[b];
    if (shapes) shapes[b] = best[b];
    if (ms) ms[b] = best_ms[b];
  }
  // the outputs of the chosen shapes (every shape gives the same results)
  Workspace ws;
  return weights_run(ctx, st, ops, n_ops, precision, idx, w, status, n_bad, ws, best, nullptr);
}
