// A2-A4: batched RBF-FD weights, one saddle-point solve per stencil.
//
// Section 3, Eq. (weights): for phi(r) = r^m (m odd) and the monomials of
// degree <= l, the weights of operator L at centre x_c are the first n
// entries of the solution of
//     [Phi P; P^T 0] [w; v] = [L phi(|x - x_j|) at x_c ; L p_q(x_c)].
// The repeated solve over all N centres is the O(n^3 N) preprocessing cost
// the paper names; stencils are independent, so one workgroup solves one
// stencil and a launch covers them all (mixed n, m, l in one launch).
//
// Per workgroup:
//  1. offsets of the stencil nodes from the centre (minimum image in x),
//     scaled by rho = the largest offset length;
//  2. assembly of [A | B] in LDS (column-major), A = [Phi P; P^T 0] of size
//     K = n + M, B = one right-hand side per operator of this PHS order
//     (Section 5.3, Eq. eqn:laplacian for Laplacian^k of r^m);
//  3. LU with partial pivoting of [A | B] (FP64, or FP32 for the
//     mixed-precision variant);
//  4. back substitution, then iterative refinement: residual b - A x with A
//     and b formed in double-double arithmetic from the FP64 node
//     coordinates (so the refinement converges to the solution of the exact
//     system, not of its FP64 rounding, which for one-sided degree-5
//     stencils differs by ~5e-10), correction through the same factors,
//     until the correction is at rounding level;
//  5. rescaling by rho^-q (q = derivative order) and the padded row write.
//
// FP64 matrix cores on gfx950 have the same peak as the FP64 vector ALUs,
// so the factorisation is written on the vector ALUs.
#include <algorithm>
#include <cmath>

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
  const int *list;  // stencils of this launch (NULL: blockIdx.x itself)
};

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

// Right-hand-side entry i of operator op in double-double.
__device__ dd rhs_entry_dd(int i, int n, int m, const WOp &op, int k, const double *xh, const double *xl,
                           const double *zh, const double *zl) {
  if (i >= n) {
    int a, b;
    mono(i - n, a, b);
    return {poly_rhs(op.kind, k, a, b), 0.0};
  }
  dd x{xh[i], xl[i]}, z{zh[i], zl[i]};
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

template <typename T>
__global__ __launch_bounds__(W_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void weights_kernel(WArgs a) {
  extern __shared__ double smem[];
  const int q = a.list ? a.list[blockIdx.x] : blockIdx.x;
  const int tid = threadIdx.x;
  const int kc = a.k_cap;
  // LDS carve-up, sized by the launch's largest system kc and operator count
  double *xs = smem;                       // [n_ops][kc] solution
  double *rs = xs + a.n_ops * kc;          // [n_ops][kc] residual / correction
  double *xi = rs + a.n_ops * kc;          // [kc] scaled x offsets (FP64)
  double *ze = xi + kc;                    // [kc] scaled z offsets (FP64)
  double *xl = ze + kc;                    // [kc] low parts of the double-double x offsets
  double *zl = xl + kc;                    // [kc] low parts of the double-double z offsets
  __shared__ double s_red[4];
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

    // 5. iterative refinement with double-double residuals
    bool converged = false;
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
            const dd aij = sys_entry_dd(i, j, n, mg, xi, xl, ze, zl);
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
        if (tid == 0) s_red[1] = (dmax <= 0x1p-48 * xmax) ? 1.0 : 0.0;
      }
      __syncthreads();
      converged = s_red[1] != 0.0;
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

// count[b] and the largest K in bucket b (kmax[b])
__global__ void bucket_count_kernel(const int *n_per, int n_max, const int *l_per, int l_uni, int nc, int *count,
                                    int *kmax) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  const int K = (n_per ? n_per[q] : n_max) + n_terms(l_per ? l_per[q] : l_uni);
  const int b = bucket_of(K);
  atomicAdd(&count[b], 1);
  atomicMax(&kmax[b], K);
}

// cursor[b] starts at bucket b's offset in `list`. Each wavefront reserves
// one run per bucket and fills it in ascending stencil order, so stencils
// that are neighbours in memory stay neighbours in a launch.
__global__ void bucket_fill_kernel(const int *n_per, int n_max, const int *l_per, int l_uni, int nc, int *cursor,
                                   int *list) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool ok = q < nc;
  const int b = ok ? bucket_of((n_per ? n_per[q] : n_max) + n_terms(l_per ? l_per[q] : l_uni)) : -1;
  for (int bb = 0; bb < NBUCKET; ++bb) {
    const uint64_t mask = __ballot(b == bb);
    if (mask == 0) continue;
    int base = 0;
    if (lane == __ffsll(static_cast<unsigned long long>(mask)) - 1) base = atomicAdd(&cursor[bb], __popcll(mask));
    base = __shfl(base, __ffsll(static_cast<unsigned long long>(mask)) - 1, 64);
    if (b == bb) list[base + __popcll(mask & ((uint64_t(1) << lane) - 1))] = q;
  }
}

// Per-stencil system size K = n + M and a count of invalid parameter sets.
__global__ void ksize_kernel(const int *n_per, int n_max, const int *l_per, int l_uni, int nc,
                             int *kmax, int *n_invalid) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  int n = n_per ? n_per[q] : n_max;
  int l = l_per ? l_per[q] : l_uni;
  if (l < 0 || l > 6 || n < 1 || n > n_max) {
    atomicAdd(n_invalid, 1);
    return;
  }
  atomicMax(kmax, n + n_terms(l));
}

__global__ void count_status_kernel(const int *status, int nc, int *counts) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  int s = status[q];
  if (s == 1) atomicAdd(&counts[0], 1);
  if (s == 2) atomicAdd(&counts[1], 1);
}

}  // namespace

int weights_run(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops, int precision,
                const int32_t *idx, double *w, int32_t *status, int32_t *n_bad) {
  hipStream_t s = ctx->stream;
  const int nc = static_cast<int>(st->n_centers);
  DevBuf d_k;
  RBFFD_HIP(ctx, d_k.alloc(4 * sizeof(int)));
  RBFFD_HIP(ctx, hipMemsetAsync(d_k.p, 0, 4 * sizeof(int), s));
  ksize_kernel<<<grid_for(nc, 256), 256, 0, s>>>(st->n_per, st->n_max, st->l_per, st->l_uniform, nc,
                                                 d_k.as<int>(), d_k.as<int>() + 1);
  RBFFD_HIP(ctx, hipGetLastError());
  int hk[2];
  RBFFD_HIP(ctx, hipMemcpyAsync(hk, d_k.p, sizeof(hk), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  if (hk[1] > 0) return rbffd_fail(ctx, RBFFD_EINVAL, "%d stencils with invalid n or l", hk[1]);
  const int kc = hk[0];
  if (kc > 128) return rbffd_fail(ctx, RBFFD_EINVAL, "system size %d above 128", kc);

  DevBuf d_status;
  int32_t *st_out = status;
  if (!st_out) {
    RBFFD_HIP(ctx, d_status.alloc(sizeof(int32_t) * nc));
    st_out = d_status.as<int32_t>();
  }
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
  // stencils bucketed by K, one launch per non-empty bucket
  DevBuf d_cnt, d_list;
  RBFFD_HIP(ctx, d_cnt.alloc(3 * NBUCKET * sizeof(int)));
  RBFFD_HIP(ctx, d_list.alloc(sizeof(int) * std::max(nc, 1)));
  RBFFD_HIP(ctx, hipMemsetAsync(d_cnt.p, 0, 3 * NBUCKET * sizeof(int), s));
  bucket_count_kernel<<<grid_for(nc, 256), 256, 0, s>>>(st->n_per, st->n_max, st->l_per, st->l_uniform, nc,
                                                        d_cnt.as<int>(), d_cnt.as<int>() + 2 * NBUCKET);
  RBFFD_HIP(ctx, hipGetLastError());
  int cnt[3 * NBUCKET];   // counts, starts, largest K
  RBFFD_HIP(ctx, hipMemcpyAsync(cnt, d_cnt.p, 3 * NBUCKET * sizeof(int), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  for (int b = 0, off = 0; b < NBUCKET; ++b) {
    cnt[NBUCKET + b] = off;  // start of bucket b
    off += cnt[b];
  }
  RBFFD_HIP(ctx, hipMemcpyAsync(d_cnt.as<int>() + NBUCKET, cnt + NBUCKET, NBUCKET * sizeof(int),
                                hipMemcpyHostToDevice, s));
  bucket_fill_kernel<<<grid_for(nc, 256), 256, 0, s>>>(st->n_per, st->n_max, st->l_per, st->l_uniform, nc,
                                                       d_cnt.as<int>() + NBUCKET, d_list.as<int>());
  RBFFD_HIP(ctx, hipGetLastError());
  int used = 0;
  for (int b = 0; b < NBUCKET; ++b) used += cnt[b] > 0;
  for (int b = 0; b < NBUCKET; ++b) {
    if (cnt[b] == 0) continue;
    const int cap = cnt[2 * NBUCKET + b];  // the bucket's largest K
    a.k_cap = cap;
    a.list = used > 1 ? d_list.as<int>() + cnt[NBUCKET + b] : nullptr;
    const size_t head = sizeof(double) * (2 * static_cast<size_t>(n_ops) * cap + 4 * static_cast<size_t>(cap));
    if (precision == RBFFD_SOLVE_FP64) {
      const size_t lds = head + sizeof(double) * static_cast<size_t>(cap) * (cap + n_ops);
      if (lds > 156 * 1024) return rbffd_fail(ctx, RBFFD_EINVAL, "system size %d too large for LDS", cap);
      RBFFD_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&weights_kernel<double>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
      weights_kernel<double><<<cnt[b], W_THREADS, lds, s>>>(a);
    } else {
      const size_t lds = head + sizeof(float) * static_cast<size_t>(cap) * (cap + n_ops);
      RBFFD_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&weights_kernel<float>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
      weights_kernel<float><<<cnt[b], W_THREADS, lds, s>>>(a);
    }
  }
  RBFFD_HIP(ctx, hipGetLastError());
  RBFFD_HIP(ctx, hipMemsetAsync(d_k.p, 0, 4 * sizeof(int), s));
  count_status_kernel<<<grid_for(nc, 256), 256, 0, s>>>(st_out, nc, d_k.as<int>());
  RBFFD_HIP(ctx, hipGetLastError());
  RBFFD_HIP(ctx, hipMemcpyAsync(hk, d_k.p, sizeof(hk), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  *n_bad = hk[1] > 0 ? -hk[1] : hk[0];
  return RBFFD_OK;
}
