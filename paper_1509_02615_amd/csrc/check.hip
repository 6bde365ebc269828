// Argument checks of the search and weights entry points on the device,
// before anything is written: a call with an invalid per-stencil parameter
// or index returns RBFFD_EINVAL with every output untouched.
//
// Section 3 fixes what a well-posed stencil system needs: an odd PHS order
// m (phi = r^m), a polynomial degree l whose M = (l + 1)(l + 2) / 2 terms do
// not outnumber the n stencil nodes; Section 5.3 needs m >= 2k + 1 for
// Laplacian^k of r^m. The library adds its own limits (m <= 15, l <= 6,
// n + M <= 128, n <= n_max).
#include "common.hpp"

namespace {

enum : int {
  BAD_CENTER = 1,
  BAD_N = 2,
  BAD_M = 4,
  BAD_L = 8,
  BAD_UNDERDETERMINED = 16,
  BAD_SIZE = 32,
  BAD_HYPERLAP = 64,
  BAD_INDEX = 128
};

struct CheckArgs {
  const int *centers;
  const int *n_per, *m_per, *l_per;
  const int *idx_in;
  int n_centers, n_nodes, n_max, m_uni, l_uni;
  int weights;
  int k_max;  // largest k of the Laplacian^k operators that take the stencil's own m (0: none)
};

// flag[0]: OR of the reasons, flag[1]: smallest bad stencil
__global__ void check_params_kernel(CheckArgs a, int *flag) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  if (q < a.n_centers) {
    const int c = a.centers ? a.centers[q] : q;
    const int n = a.n_per ? a.n_per[q] : a.n_max;
    if (c < 0 || c >= a.n_nodes) bad |= BAD_CENTER;
    if (n < 1 || n > a.n_max || n > a.n_nodes) bad |= BAD_N;
    if (a.weights) {
      const int m = a.m_per ? a.m_per[q] : a.m_uni;
      const int l = a.l_per ? a.l_per[q] : a.l_uni;
      if (m < 1 || m > 15 || (m & 1) == 0) bad |= BAD_M;
      if (l < 0 || l > 6) {
        bad |= BAD_L;
      } else {
        const int M = (l + 1) * (l + 2) / 2;
        if (n < M) bad |= BAD_UNDERDETERMINED;
        if (n + M > 128) bad |= BAD_SIZE;
      }
      if (a.k_max > 0 && m < 2 * a.k_max + 1) bad |= BAD_HYPERLAP;
    }
  }
  if (__ballot(bad != 0) == 0) return;  // the usual case: one vote per wavefront
  if (bad) {
    atomicOr(&flag[0], bad);
    atomicMin(&flag[1], q);
  }
}

// Given stencils: one thread per entry of idx_in, entries past n_q ignored.
__global__ void check_index_kernel(CheckArgs a, int *flag) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t total = static_cast<int64_t>(a.n_centers) * a.n_max;
  bool bad = false;
  int q = 0;
  if (e < total) {
    q = static_cast<int>(e / a.n_max);
    const int t = static_cast<int>(e - static_cast<int64_t>(q) * a.n_max);
    const int n = a.n_per ? a.n_per[q] : a.n_max;
    if (t < n && t < a.n_max) {
      const int j = a.idx_in[e];
      bad = j < 0 || j >= a.n_nodes;
    }
  }
  if (__ballot(bad) == 0) return;
  if (bad) {
    atomicOr(&flag[0], BAD_INDEX);
    atomicMin(&flag[1], q);
  }
}

}  // namespace

int check_stencils_device(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops, bool weights,
                          Workspace &ws) {
  CheckArgs a{};
  a.centers = st->centers;
  a.n_per = st->n_per;
  a.m_per = st->m_per;
  a.l_per = st->l_per;
  a.idx_in = weights ? st->idx_in : nullptr;
  a.n_centers = static_cast<int>(st->n_centers);
  a.n_nodes = static_cast<int>(st->n_nodes);
  a.n_max = st->n_max;
  a.m_uni = st->m_uniform;
  a.l_uni = st->l_uniform;
  a.weights = weights ? 1 : 0;
  for (int i = 0; weights && i < n_ops; ++i)  // Laplacian^k on the stencil's own m (k = 0: m's default)
    if (ops[i].kind == RBFFD_HYPERLAP && ops[i].phs_order == 0) a.k_max = std::max(a.k_max, ops[i].k);
  hipStream_t s = ctx->stream;
  int *d_flag;
  RBFFD_WS(ctx, ws, ws.get(2, &d_flag));
  const int init[2] = {0, a.n_centers};
  RBFFD_HIP(ctx, hipMemcpyAsync(d_flag, init, sizeof(init), hipMemcpyHostToDevice, s));
  check_params_kernel<<<grid_for(a.n_centers, 256), 256, 0, s>>>(a, d_flag);
  if (a.idx_in) {
    const int64_t total = static_cast<int64_t>(a.n_centers) * a.n_max;
    check_index_kernel<<<grid_for(total, 256), 256, 0, s>>>(a, d_flag);
  }
  RBFFD_HIP(ctx, hipGetLastError());
  int flag[2];
  RBFFD_HIP(ctx, hipMemcpyAsync(flag, d_flag, sizeof(flag), hipMemcpyDeviceToHost, s));
  RBFFD_HIP(ctx, hipStreamSynchronize(s));
  if (!flag[0]) return RBFFD_OK;
  const int f = flag[0];
  const char *why = (f & BAD_CENTER) ? "centre index outside the node set"
                    : (f & BAD_N) ? "stencil size outside 1..min(n_max, n_nodes)"
                    : (f & BAD_M) ? "PHS order m not odd in 1..15"
                    : (f & BAD_L) ? "polynomial degree l outside 0..6"
                    : (f & BAD_UNDERDETERMINED) ? "fewer stencil nodes than polynomial terms"
                    : (f & BAD_SIZE) ? "system size n + M above 128"
                    : (f & BAD_HYPERLAP) ? "Laplacian^k of r^m not continuous (m < 2k + 1)"
                                         : "given stencil index outside the node set";
  return rbffd_fail(ctx, RBFFD_EINVAL, "stencil %d: %s (nothing written)", flag[1], why);
}
