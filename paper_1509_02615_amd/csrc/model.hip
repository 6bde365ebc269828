// Model set-up: repack the differentiation matrices into slot-major device
// layouts, mark wall and ghost nodes, and prepare the ghost-node closure.
//
// Ghost closure (Section 5.2, Eq. bcEqn): at the boundary nodes of a wall,
// W_I u_I + W_B u_B + W_G u_G = bc, so u_G = W_G^-1 (bc - W_I u_I - W_B u_B).
// W_G (boundary rows x ghost columns, one ghost per boundary node) is a
// cyclic band matrix. It is factored once here on the host (LU with partial
// pivoting that skips structural zeros) and inverted column by column. Its
// inverse decays geometrically away from the band, so each row is stored as
// the cyclic window, centred on the row's largest entry, outside of which the
// l1 mass is below 2^-56 of the row's l1 mass: applying the window is the
// exact solve up to rounding. Each Runge-Kutta stage then applies the
// windows on the GPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "model.hpp"

namespace {

__global__ void repack_f64(const int *__restrict__ idx, const double *__restrict__ w, int64_t na, int n,
                           int *__restrict__ idx_t, RecF64 *__restrict__ rec) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= na * n) return;
  int64_t i = t / n;
  int k = static_cast<int>(t % n);
  const int64_t src = i * n + k, plane = na * n, dst = static_cast<int64_t>(k) * na + i;
  idx_t[dst] = idx[src];
  rec[dst] = RecF64{w[src], w[plane + src], w[2 * plane + src], w[3 * plane + src]};
}

__global__ void repack_f32(const int *__restrict__ idx, const double *__restrict__ w, int64_t na, int n,
                           RecF32 *__restrict__ rec, double *__restrict__ hv) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= na * n) return;
  int64_t i = t / n;
  int k = static_cast<int>(t % n);
  const int64_t src = i * n + k, plane = na * n, dst = static_cast<int64_t>(k) * na + i;
  rec[dst] = RecF32{static_cast<float>(w[src]), static_cast<float>(w[plane + src]),
                    static_cast<float>(w[2 * plane + src]), idx[src]};
  hv[dst] = w[3 * plane + src];
}

__device__ __forceinline__ uint16_t to_bf16(double v) {
  // round-to-nearest-even of the FP32 value to bfloat16 (finite inputs)
  float f = static_cast<float>(v);
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

__global__ void repack_bf16(const int *__restrict__ idx, const double *__restrict__ w, int64_t na, int n,
                            RecBF16 *__restrict__ rec, double *__restrict__ hv) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= na * n) return;
  int64_t i = t / n;
  int k = static_cast<int>(t % n);
  const int64_t src = i * n + k, plane = na * n, dst = static_cast<int64_t>(k) * na + i;
  rec[dst] = RecBF16{to_bf16(w[src]), to_bf16(w[plane + src]), to_bf16(w[2 * plane + src]), 0, idx[src]};
  hv[dst] = w[3 * plane + src];
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

__global__ void kind_kernel(uint8_t *__restrict__ kind, int64_t n_total, int64_t na, const int *__restrict__ walls,
                            int count) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n_total) kind[i] = i < na ? 0 : 2;
  // wall marks are written by a second launch of the same kernel (count > 0)
  if (count > 0 && i < count) kind[walls[i]] = 1;
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

// Half-width h of the cyclic window [c - h, c + h] around the row maximum c
// that leaves at most 2^-56 of the row's l1 mass outside. The outside mass
// is accumulated from the far end inwards (small terms first), so it is not
// the difference of two rounded sums. Returns (n - 1) / 2 + 1 when no window
// shorter than the row qualifies.
int window_halfwidth(const double *row, int n, int &center) {
  double total = 0.0, best = -1.0;
  center = 0;
  for (int j = 0; j < n; ++j) {
    double v = std::fabs(row[j]);
    total += v;
    if (v > best) {
      best = v;
      center = j;
    }
  }
  const double tol = std::ldexp(total, -56);
  const int hmax = (n - 1) / 2;
  auto at = [&](int d) { return std::fabs(row[((center + d) % n + n) % n]); };
  double tail = (n % 2 == 0) ? at(n / 2) : 0.0;  // mass at distance > hmax
  if (tail > tol) return hmax + 1;
  int h = hmax;
  while (h > 0) {
    const double next = tail + at(h) + at(-h);  // mass at distance > h - 1
    if (next > tol) break;
    tail = next;
    --h;
  }
  return h;
}

}  // namespace

static int fail_model(rbffd_ctx *ctx, rbffd_model *m, int code, const char *msg) {
  delete m;
  return rbffd_fail(ctx, code, "%s", msg);
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
  if (d->physics == RBFFD_PHYS_NS) {
    if (d->n_walls != 0 && d->n_walls != 2) return rbffd_fail(ctx, RBFFD_EINVAL, "n_walls must be 0 or 2");
    if (d->n_walls && (d->n_wall < 1 || !d->wall_nodes || !d->ghost_nodes || !d->wall_dz || !d->wall_dzz))
      return rbffd_fail(ctx, RBFFD_EINVAL, "incomplete wall description");
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

  // slot-major repack
  bool ok = true;
  if (m->physics == RBFFD_PHYS_ADVECTION) {
    ok = m->idx_t.alloc(sizeof(int) * cnt) == hipSuccess && m->rec.alloc(sizeof(RecAdv) * cnt) == hipSuccess;
    if (ok)
      repack_adv<<<grid_for(cnt, 256), 256, 0, s>>>(d->idx, d->w, d->vel_u, d->vel_v, na, m->n, m->idx_t.as<int>(),
                                                    m->rec.as<RecAdv>());
    m->bytes_per_node = n * (4 + sizeof(RecAdv));
  } else if (m->wdt == RBFFD_F64) {
    ok = m->idx_t.alloc(sizeof(int) * cnt) == hipSuccess && m->rec.alloc(sizeof(RecF64) * cnt) == hipSuccess;
    if (ok)
      repack_f64<<<grid_for(cnt, 256), 256, 0, s>>>(d->idx, d->w, na, m->n, m->idx_t.as<int>(), m->rec.as<RecF64>());
    m->bytes_per_node = n * (4 + sizeof(RecF64));
  } else if (m->wdt == RBFFD_F32) {
    ok = m->rec.alloc(sizeof(RecF32) * cnt) == hipSuccess && m->hv_t.alloc(sizeof(double) * cnt) == hipSuccess;
    if (ok) repack_f32<<<grid_for(cnt, 256), 256, 0, s>>>(d->idx, d->w, na, m->n, m->rec.as<RecF32>(), m->hv_t.as<double>());
    m->bytes_per_node = n * (sizeof(RecF32) + 8);
  } else {
    ok = m->rec.alloc(sizeof(RecBF16) * cnt) == hipSuccess && m->hv_t.alloc(sizeof(double) * cnt) == hipSuccess;
    if (ok) repack_bf16<<<grid_for(cnt, 256), 256, 0, s>>>(d->idx, d->w, na, m->n, m->rec.as<RecBF16>(), m->hv_t.as<double>());
    m->bytes_per_node = n * (sizeof(RecBF16) + 8);
  }
  if (!ok) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation (weights)");
  if (m->physics == RBFFD_PHYS_NS) {
    // own state read + base y_n read + one write per member (RK4 adds the accumulator)
    m->bytes_per_node += 8 + 1;  // pi-bar and the node kind
    if (m->pibar.alloc(sizeof(double) * na) != hipSuccess) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation");
    pibar_kernel<<<grid_for(na, 256), 256, 0, s>>>(d->xy, na, d->g / (d->c_p * d->theta_bar), m->pibar.as<double>());
  }
  if (m->kind.alloc(m->N) != hipSuccess) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation");
  kind_kernel<<<grid_for(m->N, 256), 256, 0, s>>>(m->kind.as<uint8_t>(), m->N, na, nullptr, 0);
  if (hipGetLastError() != hipSuccess) return fail_model(ctx, m, RBFFD_EDEVICE, "repack launch");

  // ghost closure
  if (m->physics == RBFFD_PHYS_NS && d->n_walls == 2) {
    const int nw = 2, nb = d->n_wall;
    m->n_walls = nw;
    m->nb = nb;
    std::vector<int> h_wall(nw * nb), h_ghost(nw * nb), h_widx(static_cast<size_t>(nw) * nb * n);
    std::vector<double> h_dz(static_cast<size_t>(nw) * nb * n), h_dzz(static_cast<size_t>(nw) * nb * n);
    if (hipMemcpyAsync(h_wall.data(), d->wall_nodes, sizeof(int) * nw * nb, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_ghost.data(), d->ghost_nodes, sizeof(int) * nw * nb, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_dz.data(), d->wall_dz, sizeof(double) * h_dz.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_dzz.data(), d->wall_dzz, sizeof(double) * h_dzz.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail_model(ctx, m, RBFFD_EDEVICE, "wall copy");
    for (int i = 0; i < nw * nb; ++i) {
      if (h_wall[i] < 0 || h_wall[i] >= na) return fail_model(ctx, m, RBFFD_EINVAL, "wall node not active");
      if (h_ghost[i] < na || h_ghost[i] >= m->N) return fail_model(ctx, m, RBFFD_EINVAL, "ghost node index not a ghost");
      if (hipMemcpyAsync(&h_widx[static_cast<size_t>(i) * n], d->idx + static_cast<int64_t>(h_wall[i]) * n,
                         sizeof(int) * n, hipMemcpyDeviceToHost, s) != hipSuccess)
        return fail_model(ctx, m, RBFFD_EDEVICE, "wall stencil copy");
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail_model(ctx, m, RBFFD_EDEVICE, "wall stencil copy");
    // ghost position per wall; W_G rows = boundary positions, columns = ghost positions
    std::vector<int> gpos(m->N - na, -1), gwall(m->N - na, -1);
    for (int wl = 0; wl < nw; ++wl)
      for (int p = 0; p < nb; ++p) {
        int gi = h_ghost[wl * nb + p] - static_cast<int>(na);
        if (gwall[gi] >= 0) return fail_model(ctx, m, RBFFD_EINVAL, "ghost node listed twice");
        gpos[gi] = p;
        gwall[gi] = wl;
      }
    std::vector<double> h_ww(static_cast<size_t>(nw) * nb * n * 2);
    std::vector<std::vector<double>> inv(nw * 2);
    int half = 0;
    std::vector<int> centers(nw * 2 * nb);
    for (int wl = 0; wl < nw; ++wl) {
      for (int op = 0; op < 2; ++op) {
        const std::vector<double> &W = op == 0 ? h_dz : h_dzz;
        std::vector<double> G(static_cast<size_t>(nb) * nb, 0.0);
        for (int b = 0; b < nb; ++b)
          for (int k = 0; k < n; ++k) {
            size_t e = (static_cast<size_t>(wl) * nb + b) * n + k;
            int j = h_widx[e];
            if (j >= na) {
              int gi = j - static_cast<int>(na);
              if (gwall[gi] != wl) return fail_model(ctx, m, RBFFD_EINVAL, "wall stencil reaches another wall's ghosts");
              G[static_cast<size_t>(b) * nb + gpos[gi]] += W[e];
            }
          }
        if (!invert_sparse_lu(nb, G, inv[wl * 2 + op]))
          return fail_model(ctx, m, RBFFD_ESINGULAR, "singular ghost block W_G");
        for (int r = 0; r < nb; ++r) {
          int c;
          int h = window_halfwidth(&inv[wl * 2 + op][static_cast<size_t>(r) * nb], nb, c);
          centers[(wl * 2 + op) * nb + r] = c;
          half = std::max(half, h);
        }
      }
      for (int b = 0; b < nb; ++b)
        for (int k = 0; k < n; ++k) {
          size_t e = (static_cast<size_t>(wl) * nb + b) * n + k;
          bool ghost = h_widx[e] >= na;
          h_ww[2 * e] = ghost ? 0.0 : h_dz[e];
          h_ww[2 * e + 1] = ghost ? 0.0 : h_dzz[e];
        }
    }
    int band = std::min(2 * half + 1, nb);
    m->band = band;
    std::vector<double> h_band(static_cast<size_t>(nw) * 2 * nb * band);
    std::vector<int> h_start(nw * 2 * nb);
    for (int mat = 0; mat < nw * 2; ++mat)
      for (int r = 0; r < nb; ++r) {
        int st = band == nb ? 0 : centers[mat * nb + r] - half;
        st = ((st % nb) + nb) % nb;
        h_start[mat * nb + r] = st;
        for (int t = 0; t < band; ++t)
          h_band[(static_cast<size_t>(mat) * nb + r) * band + t] = inv[mat][static_cast<size_t>(r) * nb + (st + t) % nb];
      }
    ok = m->wall_nodes.alloc(sizeof(int) * nw * nb) == hipSuccess &&
         m->ghost_nodes.alloc(sizeof(int) * nw * nb) == hipSuccess &&
         m->wall_idx.alloc(sizeof(int) * h_widx.size()) == hipSuccess &&
         m->wall_w.alloc(sizeof(double) * h_ww.size()) == hipSuccess &&
         m->ginv.alloc(sizeof(double) * h_band.size()) == hipSuccess &&
         m->gstart.alloc(sizeof(int) * h_start.size()) == hipSuccess &&
         m->gres.alloc(sizeof(double) * nw * nb * m->E * 4) == hipSuccess;
    if (!ok) return fail_model(ctx, m, RBFFD_ENOMEM, "device allocation (closure)");
    ok = hipMemcpy(m->wall_nodes.p, h_wall.data(), sizeof(int) * nw * nb, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->ghost_nodes.p, h_ghost.data(), sizeof(int) * nw * nb, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->wall_idx.p, h_widx.data(), sizeof(int) * h_widx.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->wall_w.p, h_ww.data(), sizeof(double) * h_ww.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->ginv.p, h_band.data(), sizeof(double) * h_band.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->gstart.p, h_start.data(), sizeof(int) * h_start.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) return fail_model(ctx, m, RBFFD_EDEVICE, "closure upload");
    kind_kernel<<<grid_for(nw * nb, 256), 256, 0, s>>>(m->kind.as<uint8_t>(), 0, na, m->wall_nodes.as<int>(), nw * nb);
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
  delete m;
  return RBFFD_OK;
}

int64_t model_bytes_per_node(rbffd_model *m) { return m->bytes_per_node; }
