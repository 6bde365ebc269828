// Model set-up: repack the differentiation matrices into slot-major device
// layouts, mark wall and ghost nodes, and prepare the ghost-node closure.
//
// Ghost closure (Section 5.2, Eq. bcEqn): at the boundary rows,
// W_I u_I + W_B u_B + W_G u_G = bc, so u_G = W_G^-1 (bc - W_I u_I - W_B u_B).
// W_G has one row per boundary row and one column per ghost; there are three
// of them (the operators applied to u, to w, and to theta' and pi'). The rows
// split into groups that share no ghost (the two walls of a channel; the
// whole perimeter of a closed box, whose corner rows couple two walls); each
// group's block is factored once here on the host (LU with partial pivoting
// that skips structural zeros) and inverted column by column. The inverse
// decays geometrically away from a row's own ghost, so each inverse row keeps
// only its entries above a cut-off chosen so that the dropped l1 mass is
// below 2^-56 of the row's l1 mass: applying the kept entries is the exact
// solve up to rounding. They are stored as the shortest cyclic window of the
// group's rows that holds them all (for a channel wall, a band around the
// row's own position), so the GPU finds each entry's row by arithmetic.
// Each Runge-Kutta stage applies the windows.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>

#include "model.hpp"

namespace {

// 16-bit offset j - i of a neighbour, or OFF_FAR
__device__ __forceinline__ int16_t nb_offset(int j, int64_t i) {
  const int64_t d = static_cast<int64_t>(j) - i;
  return (d >= -32767 && d <= 32767) ? static_cast<int16_t>(d) : OFF_FAR;
}

__global__ void repack_f64(const int *__restrict__ idx, const double *__restrict__ w, int64_t na, int n, int k0,
                           int *__restrict__ idx_t, int16_t *__restrict__ off, RecF64 *__restrict__ rec) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= na * n) return;
  int64_t i = t / n;
  int k = static_cast<int>(t % n);
  const int64_t src = i * n + k, plane = na * n, dst = static_cast<int64_t>(k - k0) * na + i;
  idx_t[static_cast<int64_t>(k) * na + i] = idx[src];
  if (k < k0) return;  // the centre slot: every centre-subtracted sum skips it
  off[dst] = nb_offset(idx[src], i);
  rec[dst] = RecF64{w[src], w[plane + src], w[2 * plane + src], w[3 * plane + src]};
}

// Signed correction q of the FP32 rounding hi of w on a grid of `scale`
// (relative), clamped to `bits` bits: w ~ hi (1 + q scale). |w - hi| <= 2^-24
// |hi| and w - hi is exact in FP64. No correction for a zero or subnormal hi.
__device__ __forceinline__ int rel_q(double w, double hi, double inv_scale, int bits) {
  if (!(fabs(hi) >= static_cast<double>(FLT_MIN))) return 0;
  const int lim = (1 << (bits - 1)) - 1;
  const int q = static_cast<int>(rint((w - hi) / hi * inv_scale));
  return max(-lim - 1, min(lim, q));
}

// FP32 rounding of a Lap^k weight, which must lie in the FP32 normal range
// (else *bad is set): the stage kernel's Lap^k sums run in FP64 on
// hi (1 + q scale).
__device__ __forceinline__ float hv_hi(double hv, int *bad) {
  const float hi = static_cast<float>(hv);
  if (hv != 0.0 && !(fabsf(hi) >= FLT_MIN && fabsf(hi) <= FLT_MAX)) atomicOr(bad, 1);
  return hi;
}

__global__ void repack_f32(const int *__restrict__ idx, const double *__restrict__ w, int64_t na, int n, int k0,
                           int *__restrict__ idx_t, uint32_t *__restrict__ aux, RecF32 *__restrict__ rec,
                           int *__restrict__ bad) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= na * n) return;
  int64_t i = t / n;
  int k = static_cast<int>(t % n);
  const int64_t src = i * n + k, plane = na * n, dst = static_cast<int64_t>(k - k0) * na + i;
  idx_t[static_cast<int64_t>(k) * na + i] = idx[src];
  if (k < k0) return;  // the centre slot: every centre-subtracted sum skips it
  const double wx = w[src], wz = w[plane + src], hv = w[3 * plane + src];
  const float hx = static_cast<float>(wx), hz = static_cast<float>(wz), hh = hv_hi(hv, bad);
  const int qh = rel_q(hv, hh, 1.0 / HV_Q_SCALE, HV_Q_BITS);
  const int qx = rel_q(wx, hx, 1.0 / D_Q_SCALE, D_Q_BITS), qz = rel_q(wz, hz, 1.0 / D_Q_SCALE, D_Q_BITS);
  rec[dst] = RecF32{hx, hz, static_cast<float>(w[2 * plane + src]), hh};
  aux[dst] = (static_cast<uint32_t>(static_cast<uint16_t>(nb_offset(idx[src], i))) << 16) |
             ((static_cast<uint32_t>(qh) & 63u) << 10) | ((static_cast<uint32_t>(qx) & 31u) << 5) |
             (static_cast<uint32_t>(qz) & 31u);
}

__global__ void repack_mw(const int *__restrict__ idx, const double *__restrict__ w, int64_t na, int n, int k0,
                          int *__restrict__ idx_t, RecMW *__restrict__ rec) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= na * n) return;
  int64_t i = t / n;
  int k = static_cast<int>(t % n);
  const int64_t src = i * n + k, plane = na * n, dst = static_cast<int64_t>(k - k0) * na + i;
  idx_t[static_cast<int64_t>(k) * na + i] = idx[src];
  if (k < k0) return;  // the centre slot: every centre-subtracted sum skips it
  rec[dst] = RecMW{w[src], w[plane + src], w[3 * plane + src], static_cast<float>(w[2 * plane + src]), idx[src]};
}

// Records of a traversal order: out[k][t] = rec[k][order[t]], copied in
// 16-byte units (`units` per record), so that the traversal reads them in
// sequence.
__global__ void permute_records(const uint4 *__restrict__ rec, const int *__restrict__ order, int64_t na, int units,
                                int64_t n_slots, uint4 *__restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_slots * na * units) return;
  const int u = static_cast<int>(t % units);
  const int64_t rest = t / units, li = rest % na, k = rest / na;
  out[(k * na + li) * units + u] = rec[(k * na + order[li]) * units + u];
}

__device__ __forceinline__ uint16_t to_bf16(double v) {
  // round-to-nearest-even of the FP32 value to bfloat16 (finite inputs)
  float f = static_cast<float>(v);
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// 8-bit correction of a bfloat16 weight b: w ~ b (1 + q 2^-15)
__device__ __forceinline__ int8_t bf_q(double w, uint16_t b) {
  const double hb = static_cast<double>(__uint_as_float(static_cast<uint32_t>(b) << 16));
  if (!(fabs(hb) >= static_cast<double>(FLT_MIN))) return 0;
  const int q = static_cast<int>(rint((w - hb) / hb * 0x1p15));
  return static_cast<int8_t>(max(-127, min(127, q)));
}

__global__ void repack_bf16(const int *__restrict__ idx, const double *__restrict__ w, int64_t na, int n, int k0,
                            int *__restrict__ idx_t, RecBF16 *__restrict__ rec, RecBF16X *__restrict__ rec2,
                            int *__restrict__ bad) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= na * n) return;
  int64_t i = t / n;
  int k = static_cast<int>(t % n);
  const int64_t src = i * n + k, plane = na * n, dst = static_cast<int64_t>(k - k0) * na + i;
  idx_t[static_cast<int64_t>(k) * na + i] = idx[src];
  if (k < k0) return;  // the centre slot: every centre-subtracted sum skips it
  const double wx = w[src], wz = w[plane + src], hv = w[3 * plane + src];
  const double wl = w[2 * plane + src];
  const uint16_t bx = to_bf16(wx), bz = to_bf16(wz), bl = to_bf16(wl);
  rec[dst] = RecBF16{bx, bz, bl, nb_offset(idx[src], i)};
  const float hh = hv_hi(hv, bad);
  rec2[dst] = RecBF16X{hh, static_cast<int8_t>(rel_q(hv, hh, 1.0 / HV_Q8_SCALE, 8)), bf_q(wl, bl), bf_q(wx, bx),
                       bf_q(wz, bz)};
}

// Transport, flux form (Section 6.1): (D_x (U psi) + D_z (V psi))_i
//   = sum_k (Wx_ik U_j + Wz_ik V_j) psi_j,  j = idx_ik.
__global__ void repack_adv(const int *__restrict__ idx, const double *__restrict__ w, const double *__restrict__ U,
                           const double *__restrict__ V, int64_t na, int n, int *__restrict__ idx_t,
                           RecAdv *__restrict__ rec) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= na * n) return;
  int64_t i = t / n;
  int k = static_cast<int>(t % n);
  const int64_t src = i * n + k, plane = na * n, dst = static_cast<int64_t>(k) * na + i;
  const int j = idx[src];
  idx_t[dst] = j;
  rec[dst] = RecAdv{w[src] * U[j] + w[plane + src] * V[j], w[2 * plane + src]};
}

// out[r][k] = idx[rows[r]][k]: rows of a row-major [.][n] index array
__global__ void gather_rows_kernel(const int *__restrict__ idx, const int *__restrict__ rows, int R, int n,
                                   int *__restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<int64_t>(R) * n) return;
  const int64_t r = t / n;
  out[t] = idx[static_cast<int64_t>(rows[r]) * n + (t - r * n)];
}

// Clears *first unless every node's stencil starts with the node itself.
__global__ void centre_first_kernel(const int *__restrict__ idx, int64_t na, int n, int *__restrict__ first) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < na && idx[i * n] != i) atomicAnd(first, 0);
}

__global__ void check_idx(const int *__restrict__ idx, int64_t count, int64_t n_total, int *__restrict__ bad) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= count) return;
  int j = idx[t];
  if (j < 0 || j >= n_total) atomicOr(bad, 1);
}

__global__ void pibar_kernel(const double *__restrict__ xy, int64_t na, double gk, double *__restrict__ pb) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < na) pb[i] = 1.0 - gk * xy[2 * i + 1];
}

// KIND_REACH on every active node with a ghost (index >= na) in its stencil
// (idx_t slot-major, [n][na]).
__global__ void reach_kernel(const int *__restrict__ idx_t, int64_t na, int n, uint8_t *__restrict__ kind) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= na) return;
  bool reach = false;
  for (int k = 0; k < n; ++k) reach |= idx_t[static_cast<int64_t>(k) * na + i] >= na;
  if (reach) kind[i] |= KIND_REACH;
}

__global__ void kind_kernel(uint8_t *__restrict__ kind, int64_t n_total, int64_t na) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n_total) kind[i] = i < na ? 0 : KIND_GHOST;
}

// ---- host-side ghost block factorisation ---------------------------------

// Dense LU with partial pivoting of an n x n row-major matrix that skips
// structural zeros, then the explicit inverse. Returns false if singular.
bool invert_sparse_lu(int n, std::vector<double> &A, std::vector<double> &inv) {
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  double amax = 0.0;
  for (double v : A) amax = std::max(amax, std::fabs(v));
  if (!(amax > 0.0)) return false;
  std::vector<int> cols, rows;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A[static_cast<size_t>(k) * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = std::fabs(A[static_cast<size_t>(i) * n + k]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    if (!(best > 1e-14 * amax)) return false;
    if (p != k) {
      std::swap_ranges(A.begin() + static_cast<size_t>(k) * n, A.begin() + static_cast<size_t>(k + 1) * n,
                       A.begin() + static_cast<size_t>(p) * n);
      std::swap(perm[k], perm[p]);
    }
    const double *pr = &A[static_cast<size_t>(k) * n];
    cols.clear();
    for (int j = k + 1; j < n; ++j)
      if (pr[j] != 0.0) cols.push_back(j);
    for (int i = k + 1; i < n; ++i) {
      double *ri = &A[static_cast<size_t>(i) * n];
      if (ri[k] == 0.0) continue;
      const double l = ri[k] / pr[k];
      ri[k] = l;
      for (int j : cols) ri[j] -= l * pr[j];
    }
  }
  // sparse lists of L (by column) and U (by row)
  std::vector<std::vector<std::pair<int, double>>> Lc(n), Ur(n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = A[static_cast<size_t>(i) * n + j];
      if (v == 0.0) continue;
      if (j < i)
        Lc[j].push_back({i, v});
      else if (j > i)
        Ur[i].push_back({j, v});
    }
  inv.assign(static_cast<size_t>(n) * n, 0.0);
  std::vector<double> y(n);
  for (int c = 0; c < n; ++c) {  // column c of A^-1: solve L U x = P e_c
    for (int i = 0; i < n; ++i) y[i] = perm[i] == c ? 1.0 : 0.0;
    for (int k = 0; k < n; ++k) {
      if (y[k] == 0.0) continue;
      for (auto &e : Lc[k]) y[e.first] -= e.second * y[k];
    }
    for (int k = n - 1; k >= 0; --k) {
      double s = y[k];
      for (auto &e : Ur[k]) s -= e.second * y[e.first];
      y[k] = s / A[static_cast<size_t>(k) * n + k];
    }
    for (int i = 0; i < n; ++i) inv[static_cast<size_t>(i) * n + c] = y[i];
  }
  for (double v : inv)
    if (!std::isfinite(v)) return false;
  return true;
}

// Indices of the entries of `row` (length n) to keep: all but the smallest
// ones whose l1 mass stays below 2^-56 of the row's l1 mass. The dropped
// mass is accumulated smallest first, so it is not the difference of two
// rounded sums. Returned in increasing index order.
std::vector<int> certified_support(const double *row, int n) {
  std::vector<int> order(n);
  for (int j = 0; j < n; ++j) order[j] = j;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return std::fabs(row[a]) < std::fabs(row[b]); });
  double total = 0.0;
  for (int j : order) total += std::fabs(row[j]);
  const double tol = std::ldexp(total, -56);
  double dropped = 0.0;
  int first = 0;
  while (first < n && dropped + std::fabs(row[order[first]]) <= tol) dropped += std::fabs(row[order[first++]]);
  std::vector<int> keep(order.begin() + first, order.end());
  std::sort(keep.begin(), keep.end());
  return keep;
}

// Shortest cyclic window [start, start + len) of 0..n-1 that holds every
// index in `keep` (sorted, non-empty): the complement of the largest gap.
void cyclic_window(const std::vector<int> &keep, int n, int &start, int &len) {
  int best_gap = -1, after = keep[0];
  for (size_t i = 0; i < keep.size(); ++i) {
    const int a = keep[i], b = i + 1 < keep.size() ? keep[i + 1] : keep[0] + n;
    if (b - a - 1 > best_gap) {
      best_gap = b - a - 1;
      after = b % n;
    }
  }
  start = after;
  len = n - best_gap;
}

int find_root(std::vector<int> &parent, int x) {
  while (parent[x] != x) x = parent[x] = parent[parent[x]];
  return x;
}

}  // namespace

static int fail_model(rbffd_ctx *ctx, rbffd_model *m, int code, const char *msg) {
  delete m;
  return rbffd_fail(ctx, code, "%s", msg);
}

// A traversal order for the member-wavefront stage kernel (ensembles of 64k
// members, where a node's member vector is 1 KiB per 64 members): the active
// nodes in Morton (Z) order of their coordinates, so that the nodes one XCD
// works on at a time form a compact patch whose neighbours' member vectors
// stay in its L2 instead of being fetched again for every stencil that
// reaches them (row-major order spans several full rows per patch, and on
// the 2048 x 256 channel at 64 members fetches a few times more bytes past
// L2 than this order). FP32 ensemble
// records are also kept in this order, so that the traversal reads them in
// sequence. The tuner keeps the order only where it is faster: it adds a
// dependent load before each wavefront's first.
static int build_order(rbffd_ctx *ctx, rbffd_model *m, const double *xy_dev) {
  const int64_t na = m->Na;
  std::vector<double> xy(static_cast<size_t>(2 * na));
  if (hipMemcpy(xy.data(), xy_dev, sizeof(double) * 2 * na, hipMemcpyDeviceToHost) != hipSuccess)
    return RBFFD_EDEVICE;
  double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
  for (int64_t i = 0; i < na; ++i)
    for (int c = 0; c < 2; ++c) {
      lo[c] = std::min(lo[c], xy[2 * i + c]);
      hi[c] = std::max(hi[c], xy[2 * i + c]);
    }
  std::vector<std::pair<uint32_t, int>> key(static_cast<size_t>(na));
  for (int64_t i = 0; i < na; ++i) {
    uint32_t code = 0;
    for (int c = 0; c < 2; ++c) {
      const double span = hi[c] > lo[c] ? hi[c] - lo[c] : 1.0;
      const uint32_t v = static_cast<uint32_t>(std::min(65535.0, std::max(0.0, (xy[2 * i + c] - lo[c]) / span * 65535.0)));
      for (int b = 0; b < 16; ++b) code |= ((v >> b) & 1u) << (2 * b + c);
    }
    key[static_cast<size_t>(i)] = {code, static_cast<int>(i)};
  }
  std::sort(key.begin(), key.end());
  std::vector<int> order(static_cast<size_t>(na));
  for (int64_t i = 0; i < na; ++i) order[static_cast<size_t>(i)] = key[static_cast<size_t>(i)].second;
  if (m->order.alloc(sizeof(int) * na) != hipSuccess) return RBFFD_ENOMEM;
  if (hipMemcpy(m->order.p, order.data(), sizeof(int) * na, hipMemcpyHostToDevice) != hipSuccess) return RBFFD_EDEVICE;
  (void)ctx;
  return RBFFD_OK;
}

int model_create_impl(rbffd_ctx *ctx, const rbffd_model_desc *d, rbffd_model **out) {
  hipStream_t s = ctx->stream;
  if (d->physics != RBFFD_PHYS_ADVECTION && d->physics != RBFFD_PHYS_NS)
    return rbffd_fail(ctx, RBFFD_EINVAL, "unknown physics %d", d->physics);
  if (d->field_dtype != RBFFD_F64 && d->field_dtype != RBFFD_F32)
    return rbffd_fail(ctx, RBFFD_EINVAL, "field dtype must be F64 or F32");
  if (d->weight_dtype < RBFFD_F64 || d->weight_dtype > RBFFD_BF16)
    return rbffd_fail(ctx, RBFFD_EINVAL, "bad weight dtype");
  if (d->weight_dtype != RBFFD_F64 && d->field_dtype != RBFFD_F32)
    return rbffd_fail(ctx, RBFFD_EINVAL, "FP32/BF16 weights need FP32 fields");
  if (d->physics == RBFFD_PHYS_ADVECTION && d->weight_dtype != RBFFD_F64)
    return rbffd_fail(ctx, RBFFD_EINVAL, "transport models keep FP64 weights");
  if (d->n < 1 || d->n > 120 || d->n_active < 1 || d->n_total < d->n_active || d->n_total >= (int64_t(1) << 31))
    return rbffd_fail(ctx, RBFFD_EINVAL, "bad sizes n=%d n_active=%lld n_total=%lld", d->n,
                      (long long)d->n_active, (long long)d->n_total);
  if (d->ensemble < 1 || d->ensemble > 4096) return rbffd_fail(ctx, RBFFD_EINVAL, "bad ensemble size");
  if (!d->idx || !d->w || !d->xy) return rbffd_fail(ctx, RBFFD_EINVAL, "null idx, w or xy");
  if (d->physics == RBFFD_PHYS_ADVECTION && (!d->vel_u || !d->vel_v || !(d->vel_period != 0.0)))
    return rbffd_fail(ctx, RBFFD_EINVAL, "transport needs vel_u, vel_v and vel_period");
  if (d->physics == RBFFD_PHYS_ADVECTION && d->n_total > d->n_active && !d->mirror_src)
    return rbffd_fail(ctx, RBFFD_EINVAL, "transport nodes past n_active need mirror_src");
  if (d->physics == RBFFD_PHYS_NS) {
    if (d->n_bnd < 0) return rbffd_fail(ctx, RBFFD_EINVAL, "n_bnd must be >= 0");
    if (d->n_bnd && (!d->bnd_nodes || !d->bnd_ghosts || !d->bnd_normal || !d->bnd_d1 || !d->bnd_d2))
      return rbffd_fail(ctx, RBFFD_EINVAL, "incomplete boundary-row description");
    if (static_cast<int64_t>(d->n_bnd) != d->n_total - d->n_active)
      return rbffd_fail(ctx, RBFFD_EINVAL, "every node past n_active must be the ghost of one boundary row");
    if (!(d->c_p > 0 && d->c_v > 0 && d->theta_bar > 0))
      return rbffd_fail(ctx, RBFFD_EINVAL, "bad physical constants");
  }

  auto *m = new (std::nothrow) rbffd_model();
  if (!m) return rbffd_fail(ctx, RBFFD_ENOMEM, "host allocation");
  m->ctx = ctx;
  m->physics = d->physics;
  m->fdt = d->field_dtype;
  m->wdt = d->weight_dtype;
  m->n = d->n;
  m->E = d->ensemble;
  m->F = d->physics == RBFFD_PHYS_NS ? 4 : 1;
  m->N = d->n_total;
  m->Na = d->n_active;
  m->hv_coeff = d->hv_coeff;
  m->vel_period = d->vel_period;
  m->c_p = d->c_p;
  m->c_v = d->c_v;
  m->R_d = d->R_d;
  m->g = d->g;
  m->theta_bar = d->theta_bar;
  m->mu = d->mu;
  m->u_bar = d->u_bar;
  const int64_t na = m->Na, n = m->n, cnt = na * n;

  // stencil indices must address existing nodes
  {
    DevBuf bad;
    if (bad.alloc(sizeof(int)) != hipSuccess) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation");
    int hb = 0;
    if (hipMemsetAsync(bad.p, 0, sizeof(int), s) != hipSuccess) return fail_model(ctx, m, RBFFD_EDEVICE, "memset");
    check_idx<<<grid_for(cnt, 256), 256, 0, s>>>(d->idx, cnt, m->N, bad.as<int>());
    if (hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail_model(ctx, m, RBFFD_EDEVICE, "index check");
    if (hb) return fail_model(ctx, m, RBFFD_EINVAL, "stencil index outside the node set");
  }

  // Navier-Stokes sums are centre-subtracted, so a centre slot adds exactly
  // 0: when every stencil starts with its own node, the stream leaves that
  // slot out (the full index array keeps it)
  if (m->physics == RBFFD_PHYS_NS && n > 1) {
    DevBuf first;
    int hf = 0;
    if (first.alloc(sizeof(int)) != hipSuccess) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation");
    if (hipMemsetAsync(first.p, 0xff, sizeof(int), s) != hipSuccess) return fail_model(ctx, m, RBFFD_EDEVICE, "memset");
    centre_first_kernel<<<grid_for(na, 256), 256, 0, s>>>(d->idx, na, m->n, first.as<int>());
    if (hipMemcpyAsync(&hf, first.p, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail_model(ctx, m, RBFFD_EDEVICE, "stencil centre check");
    m->k0 = hf ? 1 : 0;
  }
  const int k0 = m->k0;
  const int64_t cs = (n - k0) * na;  // stream records

  // slot-major repack
  bool ok = true;
  if (m->physics == RBFFD_PHYS_ADVECTION) {
    ok = m->idx_t.alloc(sizeof(int) * cnt) == hipSuccess && m->rec.alloc(sizeof(RecAdv) * cnt) == hipSuccess;
    if (ok)
      repack_adv<<<grid_for(cnt, 256), 256, 0, s>>>(d->idx, d->w, d->vel_u, d->vel_v, na, m->n, m->idx_t.as<int>(),
                                                    m->rec.as<RecAdv>());
    m->bytes_per_node = n * (4 + sizeof(RecAdv));
  } else if (m->wdt == RBFFD_F64) {
    // bytes the stage kernel streams per node: records, offsets, Lap^k
    // weights (the full indices are read only for OFF_FAR neighbours); the
    // offsets get one spare element, as a wave-uniform read takes the
    // aligned dword around an offset
    ok = m->idx_t.alloc(sizeof(int) * cnt) == hipSuccess && m->off16.alloc(sizeof(int16_t) * (cs + 1)) == hipSuccess &&
         m->rec.alloc(sizeof(RecF64) * cs) == hipSuccess;
    if (ok)
      repack_f64<<<grid_for(cnt, 256), 256, 0, s>>>(d->idx, d->w, na, m->n, k0, m->idx_t.as<int>(), m->off16.as<int16_t>(),
                                                     m->rec.as<RecF64>());
    m->bytes_per_node = (n - k0) * (sizeof(int16_t) + sizeof(RecF64));
  } else if (m->wdt == RBFFD_F32 && m->E % 64 == 0) {
    m->wide_rec = true;
    ok = m->idx_t.alloc(sizeof(int) * cnt) == hipSuccess && m->rec.alloc(sizeof(RecMW) * cs) == hipSuccess;
    if (ok)
      repack_mw<<<grid_for(cnt, 256), 256, 0, s>>>(d->idx, d->w, na, m->n, k0, m->idx_t.as<int>(), m->rec.as<RecMW>());
    m->bytes_per_node = (n - k0) * sizeof(RecMW);
  } else {
    const bool f32 = m->wdt == RBFFD_F32;
    DevBuf bad;
    ok = m->idx_t.alloc(sizeof(int) * cnt) == hipSuccess && bad.alloc(sizeof(int)) == hipSuccess &&
         (f32 ? m->aux32.alloc(sizeof(uint32_t) * cs) == hipSuccess && m->rec.alloc(sizeof(RecF32) * cs) == hipSuccess
              : m->rec.alloc(sizeof(RecBF16) * cs) == hipSuccess && m->rec2.alloc(sizeof(RecBF16X) * cs) == hipSuccess);
    if (ok) {
      int hb = 0;
      if (hipMemsetAsync(bad.p, 0, sizeof(int), s) != hipSuccess) return fail_model(ctx, m, RBFFD_EDEVICE, "memset");
      if (f32)
        repack_f32<<<grid_for(cnt, 256), 256, 0, s>>>(d->idx, d->w, na, m->n, k0, m->idx_t.as<int>(),
                                                       m->aux32.as<uint32_t>(), m->rec.as<RecF32>(), bad.as<int>());
      else
        repack_bf16<<<grid_for(cnt, 256), 256, 0, s>>>(d->idx, d->w, na, m->n, k0, m->idx_t.as<int>(),
                                                        m->rec.as<RecBF16>(), m->rec2.as<RecBF16X>(), bad.as<int>());
      if (hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail_model(ctx, m, RBFFD_EDEVICE, "weight repack");
      if (hb)
        return fail_model(ctx, m, RBFFD_EINVAL,
                          "hyperviscosity weights outside the FP32 normal range: use FP64 weights for this node set");
    }
    m->bytes_per_node = (n - k0) * (f32 ? sizeof(RecF32) + sizeof(uint32_t) : sizeof(RecBF16) + sizeof(RecBF16X));
  }
  if (!ok) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation (weights)");
  if (m->physics == RBFFD_PHYS_NS) {
    // own state read + base y_n read + one write per member (RK4 adds the accumulator)
    m->bytes_per_node += 8 + 1;  // pi-bar and the node kind
    if (m->pibar.alloc(sizeof(double) * na) != hipSuccess) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation");
    pibar_kernel<<<grid_for(na, 256), 256, 0, s>>>(d->xy, na, d->g / (d->c_p * d->theta_bar), m->pibar.as<double>());
  }
  if (m->physics == RBFFD_PHYS_NS && m->E % 64 == 0) {
    const int rc = build_order(ctx, m, d->xy);
    if (rc) return fail_model(ctx, m, rc, "traversal order");
    if (m->wide_rec) {  // the FP32 ensemble records once more, in that order
      const int64_t slots = m->n - k0;
      constexpr int units = sizeof(RecMW) / sizeof(uint4);
      if (m->rec_order.alloc(sizeof(RecMW) * slots * na) != hipSuccess)
        return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation (ordered records)");
      permute_records<<<grid_for(slots * na * units, 256), 256, 0, s>>>(m->rec.as<uint4>(), m->order.as<int>(), na, units,
                                                                         slots, m->rec_order.as<uint4>());
    }
  }
  if (m->kind.alloc(m->N) != hipSuccess) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation");
  kind_kernel<<<grid_for(m->N, 256), 256, 0, s>>>(m->kind.as<uint8_t>(), m->N, na);
  if (hipGetLastError() != hipSuccess) return fail_model(ctx, m, RBFFD_EDEVICE, "repack launch");

  // transport mirror ghosts: sources must be active nodes
  if (m->physics == RBFFD_PHYS_ADVECTION && m->N > na) {
    const int64_t ng = m->N - na;
    std::vector<int> h_src(ng);
    if (hipMemcpyAsync(h_src.data(), d->mirror_src, sizeof(int) * ng, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail_model(ctx, m, RBFFD_EDEVICE, "mirror source copy");
    for (int v : h_src)
      if (v < 0 || v >= na) return fail_model(ctx, m, RBFFD_EINVAL, "mirror source not an active node");
    if (m->mirror_src.alloc(sizeof(int) * ng) != hipSuccess) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation");
    if (hipMemcpy(m->mirror_src.p, h_src.data(), sizeof(int) * ng, hipMemcpyHostToDevice) != hipSuccess)
      return fail_model(ctx, m, RBFFD_EDEVICE, "mirror source upload");
    // the same map from the sources' side, so that a stage can write each
    // updated value into its ghosts as well
    std::vector<int> h_off(static_cast<size_t>(na) + 1, 0), h_list(static_cast<size_t>(ng));
    for (int v : h_src) ++h_off[static_cast<size_t>(v) + 1];
    for (int64_t i = 0; i < na; ++i) h_off[i + 1] += h_off[i];
    {
      std::vector<int> fill(h_off.begin(), h_off.end() - 1);
      for (int64_t k = 0; k < ng; ++k) h_list[fill[h_src[k]]++] = static_cast<int>(k);
    }
    if (m->mirror_off.alloc(sizeof(int) * h_off.size()) != hipSuccess ||
        m->mirror_list.alloc(sizeof(int) * h_list.size()) != hipSuccess)
      return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation");
    if (hipMemcpy(m->mirror_off.p, h_off.data(), sizeof(int) * h_off.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->mirror_list.p, h_list.data(), sizeof(int) * h_list.size(), hipMemcpyHostToDevice) != hipSuccess)
      return fail_model(ctx, m, RBFFD_EDEVICE, "mirror source upload");
    m->n_mirror = ng;
  }

  // ghost closure
  if (m->physics == RBFFD_PHYS_NS && d->n_bnd > 0) {
    const int R = d->n_bnd;
    m->n_bnd = R;
    std::vector<int> h_node(R), h_ghost(R), h_norm(R), h_widx(static_cast<size_t>(R) * n);
    std::vector<double> h_d1(static_cast<size_t>(R) * n), h_d2(static_cast<size_t>(R) * n);
    if (hipMemcpyAsync(h_node.data(), d->bnd_nodes, sizeof(int) * R, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_ghost.data(), d->bnd_ghosts, sizeof(int) * R, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_norm.data(), d->bnd_normal, sizeof(int) * R, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_d1.data(), d->bnd_d1, sizeof(double) * h_d1.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_d2.data(), d->bnd_d2, sizeof(double) * h_d2.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail_model(ctx, m, RBFFD_EDEVICE, "boundary-row copy");
    std::vector<int> gcol(R, -1);  // ghost (index - na) -> its row
    for (int r = 0; r < R; ++r) {
      if (h_node[r] < 0 || h_node[r] >= na) return fail_model(ctx, m, RBFFD_EINVAL, "boundary node not active");
      if (h_ghost[r] < na || h_ghost[r] >= m->N) return fail_model(ctx, m, RBFFD_EINVAL, "ghost index not a ghost");
      if (h_norm[r] != 0 && h_norm[r] != 1) return fail_model(ctx, m, RBFFD_EINVAL, "wall normal must be 0 or 1");
      int &c = gcol[h_ghost[r] - static_cast<int>(na)];
      if (c >= 0) return fail_model(ctx, m, RBFFD_EINVAL, "ghost node listed twice");
      c = r;
    }
    {  // the boundary rows' stencils: one gather on the device, one copy
      DevBuf d_rows, d_widx;
      if (d_rows.alloc(sizeof(int) * R) != hipSuccess || d_widx.alloc(sizeof(int) * h_widx.size()) != hipSuccess)
        return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation");
      const int64_t cnt_w = static_cast<int64_t>(R) * n;
      if (hipMemcpyAsync(d_rows.p, h_node.data(), sizeof(int) * R, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail_model(ctx, m, RBFFD_EDEVICE, "boundary stencil copy");
      gather_rows_kernel<<<grid_for(cnt_w, 256), 256, 0, s>>>(d->idx, d_rows.as<int>(), R, static_cast<int>(n),
                                                             d_widx.as<int>());
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(h_widx.data(), d_widx.p, sizeof(int) * h_widx.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail_model(ctx, m, RBFFD_EDEVICE, "boundary stencil copy");
    }
    // per field's operator: u takes d1 on z-normal rows and d2 on x-normal
    // rows, w the reverse, theta' and pi' d1 everywhere
    auto weight = [&](int mat, int r, int k) {
      const size_t e = static_cast<size_t>(r) * n + k;
      const bool zn = h_norm[r] == 0;
      return mat == 2 ? h_d1[e] : ((mat == 0) == zn ? h_d1[e] : h_d2[e]);
    };
    // groups of rows that share ghosts (union-find over row - ghost-column links)
    std::vector<int> parent(R);
    for (int r = 0; r < R; ++r) parent[r] = r;
    for (int r = 0; r < R; ++r)
      for (int k = 0; k < n; ++k) {
        const int j = h_widx[static_cast<size_t>(r) * n + k];
        if (j >= na) {
          const int a = find_root(parent, r), b = find_root(parent, gcol[j - static_cast<int>(na)]);
          if (a != b) parent[a] = b;
        }
      }
    std::vector<std::vector<int>> groups;
    {
      std::vector<int> gid(R, -1);
      for (int r = 0; r < R; ++r) {
        const int root = find_root(parent, r);
        if (gid[root] < 0) {
          gid[root] = static_cast<int>(groups.size());
          groups.emplace_back();
        }
        groups[gid[root]].push_back(r);
      }
    }
    // rows renumbered so each group is contiguous: group rows first, in
    // the caller's order within the group
    std::vector<int> perm;                 // new position -> caller's row
    std::vector<int> h_g0(R), h_gm(R);     // per new row: its group's first position and size
    for (const auto &grp : groups) {
      const int g0 = static_cast<int>(perm.size());
      for (int r : grp) {
        h_g0[perm.size()] = g0;
        h_gm[perm.size()] = static_cast<int>(grp.size());
        perm.push_back(r);
      }
    }
    // inverse rows of the three blocks as cyclic windows over the group
    std::vector<int> h_win(3 * static_cast<size_t>(R) * 2);     // {start, len} per (matrix, new row)
    std::vector<int64_t> h_off(3 * static_cast<size_t>(R));      // value offset per (matrix, new row)
    std::vector<double> h_val;
    std::vector<int> local(R, -1);
    for (const auto &grp : groups) {
      const int gm = static_cast<int>(grp.size());
      for (int i = 0; i < gm; ++i) local[grp[i]] = i;
      bool has_x = false;
      for (int r : grp) has_x = has_x || h_norm[r] == 1;
      std::vector<double> inv_tp;
      for (int mat : {2, 1, 0}) {
        std::vector<double> inv;
        if (mat == 0 && !has_x) {
          inv = inv_tp;  // u and theta' take the same operator on z-normal rows
        } else {
          std::vector<double> G(static_cast<size_t>(gm) * gm, 0.0);
          for (int i = 0; i < gm; ++i)
            for (int k = 0; k < n; ++k) {
              const int j = h_widx[static_cast<size_t>(grp[i]) * n + k];
              if (j >= na) G[static_cast<size_t>(i) * gm + local[gcol[j - static_cast<int>(na)]]] += weight(mat, grp[i], k);
            }
          if (!invert_sparse_lu(gm, G, inv)) return fail_model(ctx, m, RBFFD_ESINGULAR, "singular ghost block W_G");
        }
        const int g0 = h_g0[static_cast<size_t>(std::find(perm.begin(), perm.end(), grp[0]) - perm.begin())];
        for (int i = 0; i < gm; ++i) {
          const double *row = &inv[static_cast<size_t>(i) * gm];
          int st = 0, len = 0;
          cyclic_window(certified_support(row, gm), gm, st, len);
          const size_t slot = static_cast<size_t>(mat) * R + g0 + i;
          h_win[2 * slot] = st;
          h_win[2 * slot + 1] = len;
          h_off[slot] = static_cast<int64_t>(h_val.size());
          for (int q = 0; q < len; ++q) h_val.push_back(row[(st + q) % gm]);
          m->inv_max_row = std::max(m->inv_max_row, len);
        }
        if (mat == 2) inv_tp = std::move(inv);
      }
    }
    m->u_shares_tp = std::all_of(h_norm.begin(), h_norm.end(), [](int v) { return v == 0; }) ? 1 : 0;
    // per-row arrays in the new order; boundary weights with ghost entries zeroed
    std::vector<int> p_node(R), p_ghost(R), p_norm(R), p_widx(static_cast<size_t>(R) * n);
    std::vector<double> h_ww(static_cast<size_t>(R) * n * 2);
    for (int r = 0; r < R; ++r) {
      const int o = perm[r];
      p_node[r] = h_node[o];
      p_ghost[r] = h_ghost[o];
      p_norm[r] = h_norm[o];
      for (int k = 0; k < n; ++k) {
        const size_t e = static_cast<size_t>(r) * n + k, eo = static_cast<size_t>(o) * n + k;
        p_widx[e] = h_widx[eo];
        const bool ghost = h_widx[eo] >= na;
        h_ww[2 * e] = ghost ? 0.0 : h_d1[eo];
        h_ww[2 * e + 1] = ghost ? 0.0 : h_d2[eo];
      }
    }
    std::vector<uint8_t> h_kind(static_cast<size_t>(m->N), 0);
    for (int64_t i = na; i < m->N; ++i) h_kind[i] = KIND_GHOST;
    for (int r = 0; r < R; ++r) h_kind[h_node[r]] |= h_norm[r] == 0 ? KIND_ZWALL : KIND_XWALL;
    std::vector<int2> h_grp(R);
    for (int r = 0; r < R; ++r) h_grp[r] = make_int2(h_g0[r], h_gm[r]);
    ok = m->bnd_nodes.alloc(sizeof(int) * R) == hipSuccess && m->bnd_ghosts.alloc(sizeof(int) * R) == hipSuccess &&
         m->bnd_normal.alloc(sizeof(int) * R) == hipSuccess && m->wall_idx.alloc(sizeof(int) * p_widx.size()) == hipSuccess &&
         m->wall_w.alloc(sizeof(double) * h_ww.size()) == hipSuccess &&
         m->inv_grp.alloc(sizeof(int2) * R) == hipSuccess && m->inv_win.alloc(sizeof(int) * h_win.size()) == hipSuccess &&
         m->inv_off.alloc(sizeof(int64_t) * h_off.size()) == hipSuccess &&
         m->inv_val.alloc(sizeof(double) * h_val.size()) == hipSuccess &&
         m->gres.alloc(sizeof(double) * R * m->E * 4) == hipSuccess;
    if (ok && m->fdt == RBFFD_F32 && m->N > na)
      ok = m->ghrem.alloc(sizeof(float) * (m->N - na) * m->E * 4) == hipSuccess &&
           hipMemset(m->ghrem.p, 0, m->ghrem.bytes) == hipSuccess;
    if (!ok) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation (closure)");
    ok = hipMemcpy(m->bnd_nodes.p, p_node.data(), sizeof(int) * R, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->bnd_ghosts.p, p_ghost.data(), sizeof(int) * R, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->bnd_normal.p, p_norm.data(), sizeof(int) * R, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->wall_idx.p, p_widx.data(), sizeof(int) * p_widx.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->wall_w.p, h_ww.data(), sizeof(double) * h_ww.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->inv_grp.p, h_grp.data(), sizeof(int2) * R, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->inv_win.p, h_win.data(), sizeof(int) * h_win.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->inv_off.p, h_off.data(), sizeof(int64_t) * h_off.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->inv_val.p, h_val.data(), sizeof(double) * h_val.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->kind.p, h_kind.data(), static_cast<size_t>(m->N), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) return fail_model(ctx, m, RBFFD_EDEVICE, "closure upload");
    reach_kernel<<<grid_for(na, 256), 256, 0, s>>>(m->idx_t.as<int>(), na, m->n, m->kind.as<uint8_t>());
    if (hipGetLastError() != hipSuccess) return fail_model(ctx, m, RBFFD_EDEVICE, "node kinds");
  }
  // RK buffers
  const size_t sb = m->state_bytes();
  ok = m->ya.alloc(sb) == hipSuccess && m->yb.alloc(sb) == hipSuccess && m->acc.alloc(sb) == hipSuccess &&
       m->dev_misc.alloc(sizeof(DevMisc)) == hipSuccess;
  if (!ok) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation (stage buffers)");
  if (hipMemsetAsync(m->ya.p, 0, sb, s) != hipSuccess || hipMemsetAsync(m->yb.p, 0, sb, s) != hipSuccess ||
      hipMemsetAsync(m->acc.p, 0, sb, s) != hipSuccess || hipGetLastError() != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail_model(ctx, m, RBFFD_EDEVICE, "model set-up");
  *out = m;
  return RBFFD_OK;
}

int model_destroy_impl(rbffd_model *m) {
  if (!m) return RBFFD_OK;
  if (m->ctx) (void)hipSetDevice(m->ctx->device);
  for (auto &p : m->prof_events) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  if (m->exec_n) (void)hipGraphExecDestroy(m->exec_n);
  if (m->graph_n) (void)hipGraphDestroy(m->graph_n);
  delete m;
  return RBFFD_OK;
}

int64_t model_bytes_per_node(rbffd_model *m) { return m->bytes_per_node; }
