// extern "C" entry points of librbffd: argument checks and dispatch.
#include <cstdarg>
#include <mutex>
#include <new>

#include "common.hpp"

// ---- scratch of the allocation-free weights entry point ----
//
// rbffd_weights_noalloc takes its device scratch from this array instead of
// allocating. Each device holds its own copy (for as long as the process
// runs); host code never passes the array's name to a kernel or a copy --
// in host code it is only a stand-in -- but the device address that
// hipGetSymbolAddress returns for the current device, taken once per device
// by rbffd_create. The size covers the search and the weights at the
// documented limits (RBFFD_NOALLOC_MAX_NODES, RBFFD_NOALLOC_MAX_CENTERS).
namespace {
constexpr size_t NOALLOC_BYTES = CHECK_SCRATCH_BYTES +
                                 knn_scratch_bytes(RBFFD_NOALLOC_MAX_NODES, RBFFD_NOALLOC_MAX_CENTERS) +
                                 weights_scratch_bytes(RBFFD_NOALLOC_MAX_CENTERS);
}  // namespace
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on `device` (which must be current),
// looked up on first use.
hipError_t scratch_for(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

int rbffd_fail(rbffd_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return code;
}

extern "C" {

int rbffd_create(rbffd_ctx **out, int device, void *hip_stream) {
  if (!out) return RBFFD_EINVAL;
  *out = nullptr;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev)
    return RBFFD_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return RBFFD_EDEVICE;
  auto *ctx = new (std::nothrow) rbffd_ctx();
  if (!ctx) return RBFFD_ENOMEM;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->n_cu = prop.multiProcessorCount;
  // set-up of the allocation-free entry point's scratch on this device
  if (scratch_for(device, &ctx->scratch) != hipSuccess) {
    delete ctx;
    return RBFFD_EDEVICE;
  }
  *out = ctx;
  return RBFFD_OK;
}

int rbffd_destroy(rbffd_ctx *ctx) {
  delete ctx;
  return RBFFD_OK;
}

const char *rbffd_last_error(rbffd_ctx *ctx) {
  return ctx ? ctx->last_error.c_str() : "null context";
}

int rbffd_sync(rbffd_ctx *ctx) {
  if (!ctx) return RBFFD_EINVAL;
  RBFFD_ENTER(ctx);
  RBFFD_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return RBFFD_OK;
}

static int check_stencils(rbffd_ctx *ctx, const rbffd_stencils *st) {
  if (!st) return rbffd_fail(ctx, RBFFD_EINVAL, "null stencil description");
  if (st->n_nodes <= 0 || st->n_nodes >= (int64_t(1) << 31) || !st->xy)
    return rbffd_fail(ctx, RBFFD_EINVAL, "bad node set (n_nodes=%lld)", (long long)st->n_nodes);
  if (st->n_centers < 0 || st->n_centers >= (int64_t(1) << 31))
    return rbffd_fail(ctx, RBFFD_EINVAL, "bad n_centers=%lld", (long long)st->n_centers);
  if (st->n_max < 1 || st->n_max > 120)
    return rbffd_fail(ctx, RBFFD_EINVAL, "n_max=%d outside 1..120", st->n_max);
  if (st->n_max > st->n_nodes)
    return rbffd_fail(ctx, RBFFD_EINVAL, "stencil larger than the node set");
  if (!(st->period_x >= 0.0)) return rbffd_fail(ctx, RBFFD_EINVAL, "negative period");
  return RBFFD_OK;
}

int rbffd_knn(rbffd_ctx *ctx, const rbffd_stencils *st, int32_t *idx) {
  if (!ctx) return RBFFD_EINVAL;
  int rc = check_stencils(ctx, st);
  if (rc) return rc;
  if (st->n_centers == 0) return RBFFD_OK;  // empty batch: nothing to write
  if (!idx) return rbffd_fail(ctx, RBFFD_EINVAL, "null idx");
  RBFFD_ENTER(ctx);
  Workspace ws;
  rc = check_stencils_device(ctx, st, nullptr, 0, false, ws);
  if (rc) return rc;
  return knn_run(ctx, st, idx, ws);
}

// Checks of the uniform arguments of a weights call that need no device.
static int check_weights_host(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops,
                              int precision) {
  int rc = check_stencils(ctx, st);
  if (rc) return rc;
  if (!ops || n_ops < 1 || n_ops > 8) return rbffd_fail(ctx, RBFFD_EINVAL, "n_ops=%d outside 1..8", n_ops);
  if (precision != RBFFD_SOLVE_FP64 && precision != RBFFD_SOLVE_FP32_IR)
    return rbffd_fail(ctx, RBFFD_EINVAL, "bad precision %d", precision);
  // Uniform parameters are checked here; per-centre ones on the device
  // before anything is written.
  if (!st->m_per && (st->m_uniform < 1 || st->m_uniform > 15 || st->m_uniform % 2 == 0))
    return rbffd_fail(ctx, RBFFD_EINVAL, "PHS order m=%d must be odd in 1..15", st->m_uniform);
  if (!st->l_per && (st->l_uniform < 0 || st->l_uniform > 6))
    return rbffd_fail(ctx, RBFFD_EINVAL, "degree l=%d outside 0..6", st->l_uniform);
  for (int i = 0; i < n_ops; ++i) {
    const rbffd_op &o = ops[i];
    if (o.kind < RBFFD_DX || o.kind > RBFFD_DXX || o.reserved != 0 || o.k < 0 || o.k > 7 ||
        o.phs_order < 0 || o.phs_order > 15 || (o.phs_order && o.phs_order % 2 == 0))
      return rbffd_fail(ctx, RBFFD_EINVAL, "bad operator %d (kind %d k %d order %d)", i, o.kind,
                        o.k, o.phs_order);
    if (o.kind == RBFFD_HYPERLAP && o.k > 0) {
      int m = o.phs_order ? o.phs_order : (st->m_per ? 15 : st->m_uniform);
      if (m < 2 * o.k + 1)
        return rbffd_fail(ctx, RBFFD_EINVAL, "Laplacian^%d of r^%d is not continuous", o.k, m);
    }
  }
  if (!st->n_per && !st->l_per) {
    int M = (st->l_uniform + 1) * (st->l_uniform + 2) / 2;
    if (st->n_max < M)
      return rbffd_fail(ctx, RBFFD_EINVAL, "stencil size %d below the %d polynomial terms", st->n_max, M);
    if (st->n_max + M > 128)
      return rbffd_fail(ctx, RBFFD_EINVAL, "system size %d above 128", st->n_max + M);
  }
  return RBFFD_OK;
}

// A1-A4 on a workspace: device argument checks (nothing is written before
// they pass), the search (or a copy of the given stencils), then the solves
// (tuned: one run per candidate launch shape, the fastest shape per size
// bucket kept in the context).
static int weights_impl(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops, int precision,
                        int32_t *idx, double *w, int32_t *status, Workspace &ws, bool tune = false,
                        int32_t *shapes = nullptr, double *ms = nullptr) {
  int rc = check_stencils_device(ctx, st, ops, n_ops, true, ws);
  if (rc) return rc;
  const int32_t *use_idx = st->idx_in;
  if (!use_idx) {
    rc = knn_run(ctx, st, idx, ws);
    if (rc) return rc;
    use_idx = idx;
  } else if (idx) {
    RBFFD_HIP(ctx, hipMemcpyAsync(idx, st->idx_in, sizeof(int32_t) * st->n_centers * st->n_max,
                                  hipMemcpyDeviceToDevice, ctx->stream));
  }
  int32_t n_bad = 0;
  rc = tune ? weights_tune(ctx, st, ops, n_ops, precision, use_idx, w, status, &n_bad, shapes, ms)
            : weights_run(ctx, st, ops, n_ops, precision, use_idx, w, status, &n_bad, ws);
  if (rc) return rc;
  if (n_bad < 0) return rbffd_fail(ctx, RBFFD_EINVAL, "%d stencils have invalid m, l or n", -n_bad);
  if (n_bad > 0) return rbffd_fail(ctx, RBFFD_ESINGULAR, "%d singular stencil systems", n_bad);
  return RBFFD_OK;
}

int rbffd_weights(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops,
                  int precision, int32_t *idx, double *w, int32_t *status) {
  if (!ctx) return RBFFD_EINVAL;
  int rc = check_weights_host(ctx, st, ops, n_ops, precision);
  if (rc) return rc;
  if (st->n_centers == 0) return RBFFD_OK;  // empty batch: nothing to write
  if (!w) return rbffd_fail(ctx, RBFFD_EINVAL, "null w");
  if (!st->idx_in && !idx) return rbffd_fail(ctx, RBFFD_EINVAL, "need idx output or idx_in");
  RBFFD_ENTER(ctx);
  Workspace ws;
  return weights_impl(ctx, st, ops, n_ops, precision, idx, w, status, ws);
}

int rbffd_weights_tune(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops, int precision,
                       int32_t *idx, double *w, int32_t *status, int32_t *shapes, double *bucket_ms) {
  if (!ctx) return RBFFD_EINVAL;
  int rc = check_weights_host(ctx, st, ops, n_ops, precision);
  if (rc) return rc;
  if (shapes)
    for (int b = 0; b < RBFFD_WEIGHT_BUCKETS; ++b)
      if (shapes[b] < -1 || shapes[b] >= weights_shape_count(b))
        return rbffd_fail(ctx, RBFFD_EINVAL, "shape %d of bucket %d outside -1..%d", shapes[b], b,
                          weights_shape_count(b) - 1);
  if (st->n_centers == 0) return RBFFD_OK;  // empty batch: nothing to write
  if (!w) return rbffd_fail(ctx, RBFFD_EINVAL, "null w");
  if (!st->idx_in && !idx) return rbffd_fail(ctx, RBFFD_EINVAL, "need idx output or idx_in");
  RBFFD_ENTER(ctx);
  Workspace ws;
  return weights_impl(ctx, st, ops, n_ops, precision, idx, w, status, ws, true, shapes, bucket_ms);
}

int rbffd_weights_noalloc(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops,
                          int precision, int32_t *idx, double *w, int32_t *status) {
  if (!ctx) return RBFFD_EINVAL;
  int rc = check_weights_host(ctx, st, ops, n_ops, precision);
  if (rc) return rc;
  if (st->n_nodes > RBFFD_NOALLOC_MAX_NODES || st->n_centers > RBFFD_NOALLOC_MAX_CENTERS)
    return rbffd_fail(ctx, RBFFD_EINVAL, "%lld nodes / %lld centres beyond the allocation-free limits (%d / %d)",
                      (long long)st->n_nodes, (long long)st->n_centers, RBFFD_NOALLOC_MAX_NODES,
                      RBFFD_NOALLOC_MAX_CENTERS);
  if (st->n_centers == 0) return RBFFD_OK;  // empty batch: nothing to write
  if (!w) return rbffd_fail(ctx, RBFFD_EINVAL, "null w");
  if (!st->idx_in && !idx) return rbffd_fail(ctx, RBFFD_EINVAL, "need idx output or idx_in");
  if (!ctx->scratch) return rbffd_fail(ctx, RBFFD_EDEVICE, "no scratch region on device %d", ctx->device);
  RBFFD_ENTER(ctx);
  Workspace ws(ctx->scratch, NOALLOC_BYTES);
  return weights_impl(ctx, st, ops, n_ops, precision, idx, w, status, ws);
}

int rbffd_model_create(rbffd_ctx *ctx, const rbffd_model_desc *desc, rbffd_model **out) {
  if (!ctx) return RBFFD_EINVAL;
  if (!desc || !out) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  *out = nullptr;
  RBFFD_ENTER(ctx);
  return model_create_impl(ctx, desc, out);
}

int rbffd_model_destroy(rbffd_model *model) { return model_destroy_impl(model); }

int rbffd_ghost(rbffd_ctx *ctx, rbffd_model *model, void *state) {
  if (!ctx) return RBFFD_EINVAL;
  if (!model || !state) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  RBFFD_ENTER(ctx);
  return model_ghost(ctx, model, state);
}

int rbffd_rhs(rbffd_ctx *ctx, rbffd_model *model, double t, void *state, void *tendency) {
  if (!ctx) return RBFFD_EINVAL;
  if (!model || !state || !tendency) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  RBFFD_ENTER(ctx);
  return model_rhs(ctx, model, t, state, tendency);
}

int rbffd_step(rbffd_ctx *ctx, rbffd_model *model, void *state, double *t, double dt,
               int64_t n_steps, int tableau) {
  if (!ctx) return RBFFD_EINVAL;
  if (!model || !state || !t) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  if (n_steps < 0 || n_steps >= (int64_t(1) << 31))
    return rbffd_fail(ctx, RBFFD_EINVAL, "bad n_steps");
  if (tableau != RBFFD_RK4 && tableau != RBFFD_WSRK3)
    return rbffd_fail(ctx, RBFFD_EINVAL, "bad tableau %d", tableau);
  if (!(dt > 0.0)) return rbffd_fail(ctx, RBFFD_EINVAL, "dt must be positive");
  RBFFD_ENTER(ctx);
  return model_step(ctx, model, state, t, dt, n_steps, tableau);
}

int64_t rbffd_model_bytes_per_node(rbffd_model *model) {
  return model ? model_bytes_per_node(model) : 0;
}

int rbffd_model_profile(rbffd_model *model, int enable) {
  if (!model) return RBFFD_EINVAL;
  return model_profile(model, enable);
}

int rbffd_model_profile_read(rbffd_model *model, double *total_ms, int64_t *launches) {
  if (!model || !total_ms || !launches) return RBFFD_EINVAL;
  return model_profile_read(model, total_ms, launches);
}

int rbffd_model_tune(rbffd_ctx *ctx, rbffd_model *model, void *state, int *chosen, double *best_us) {
  if (!ctx) return RBFFD_EINVAL;
  if (!model || !state || !chosen || !best_us) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  RBFFD_ENTER(ctx);
  return model_tune(ctx, model, state, chosen, best_us);
}

int rbffd_closure_create(rbffd_ctx *ctx, rbffd_model *model, const rbffd_closure_desc *desc, rbffd_closure **out) {
  if (!ctx) return RBFFD_EINVAL;
  if (!model || !desc || !out) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  *out = nullptr;
  RBFFD_ENTER(ctx);
  return closure_create(ctx, model, desc, out);
}

int rbffd_closure_destroy(rbffd_closure *cl) { return closure_destroy(cl); }

float *rbffd_closure_params(rbffd_closure *cl) { return cl ? closure_params(cl) : nullptr; }

int rbffd_closure_forward(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, float *out) {
  if (!ctx) return RBFFD_EINVAL;
  if (!cl || !state || !out) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  RBFFD_ENTER(ctx);
  return closure_forward(ctx, cl, state, out);
}

int rbffd_closure_tune(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, int *chosen, double *best_us) {
  if (!ctx) return RBFFD_EINVAL;
  if (!cl || !state || !chosen || !best_us) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  RBFFD_ENTER(ctx);
  return closure_tune(ctx, cl, state, chosen, best_us);
}

int rbffd_closure_gradient(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, const float *target, float *grad,
                           double *loss) {
  if (!ctx) return RBFFD_EINVAL;
  if (!cl || !state || !target || !grad || !loss) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  RBFFD_ENTER(ctx);
  return closure_gradient(ctx, cl, state, target, grad, loss);
}

int rbffd_closure_train_step(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, const float *target, double lr,
                             double *loss) {
  if (!ctx) return RBFFD_EINVAL;
  if (!cl || !state || !target || !loss) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  if (!(lr > 0.0)) return rbffd_fail(ctx, RBFFD_EINVAL, "learning rate must be positive");
  RBFFD_ENTER(ctx);
  return closure_train_step(ctx, cl, state, target, lr, loss);
}

int rbffd_closure_step(rbffd_ctx *ctx, rbffd_closure *cl, void *state, double *t, double dt, int64_t n_steps,
                       int tableau, int64_t *n_fallback) {
  if (!ctx) return RBFFD_EINVAL;
  if (!cl || !state || !t) return rbffd_fail(ctx, RBFFD_EINVAL, "null argument");
  if (n_steps < 0 || !(dt > 0.0) || (tableau != RBFFD_RK4 && tableau != RBFFD_WSRK3))
    return rbffd_fail(ctx, RBFFD_EINVAL, "bad step arguments");
  RBFFD_ENTER(ctx);
  return closure_step(ctx, cl, state, t, dt, n_steps, tableau, n_fallback);
}

int rbffd_stream_copy(rbffd_ctx *ctx, void *dst, const void *src, int64_t bytes) {
  if (!ctx) return RBFFD_EINVAL;
  if (!dst || !src || bytes < 0 || bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 ||
      reinterpret_cast<uintptr_t>(src) % 16)
    return rbffd_fail(ctx, RBFFD_EINVAL, "stream copy needs 16-byte aligned pointers and size");
  RBFFD_ENTER(ctx);
  return stream_copy(ctx, dst, src, bytes);
}

int rbffd_mfma_probe(rbffd_ctx *ctx, int shape, float *out, int64_t n_out, int iters, int64_t *flops) {
  if (!ctx || !flops) return RBFFD_EINVAL;
  RBFFD_ENTER(ctx);
  return mfma_probe(ctx, shape, out, n_out, iters, flops);
}

}  // extern "C"
